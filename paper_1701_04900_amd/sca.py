"""Thin ctypes binding of libsca (include/sca.h): argument marshalling only.

Every function named ``sca_*`` here calls the C entry point of the same name; device
buffers are torch CUDA tensors (their data pointers are passed), streams are torch's
current HIP stream.  Nothing here computes: when libsca.so is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsca.so")

SCA_OK, SCA_EINVAL, SCA_ENOMEM, SCA_EHIP, SCA_ENONFINITE, SCA_ENOTCONV = range(6)
SCA_F32, SCA_F64 = 0, 1
SCA_REG_L1, SCA_REG_EXP, SCA_REG_LOG = 0, 1, 2
SCA_FLAG_PROFILE = 1
SCA_K_SELECT, SCA_K_GRAD, SCA_K_COMPACT, SCA_K_FOLD, SCA_K_NKINDS = range(5)
_STATUS = {0: "SCA_OK", 1: "SCA_EINVAL", 2: "SCA_ENOMEM", 3: "SCA_EHIP", 4: "SCA_ENONFINITE",
           5: "SCA_ENOTCONV"}


class SCAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class sca_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("gamma", ctypes.c_double),
                ("gamma_mu", ctypes.c_double), ("tau", ctypes.c_double),
                ("select_p", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("instance", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("max_rounds", ctypes.c_int64), ("check_every", ctypes.c_int64),
                ("refresh_every", ctypes.c_int64), ("tol_rel_obj", ctypes.c_double),
                ("F_star", ctypes.c_double), ("tol_merit", ctypes.c_double),
                ("delay_chunks", ctypes.c_int64), ("delay_stale", ctypes.c_int64),
                ("async_workgroups", ctypes.c_int64)]


class sca_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("rounds", ctypes.c_int64),
                ("coord_updates", ctypes.c_int64), ("moved_updates", ctypes.c_int64),
                ("F", ctypes.c_double),
                ("merit", ctypes.c_double), ("MF", ctypes.c_double),
                ("rel_err", ctypes.c_double), ("seconds", ctypes.c_double),
                ("nnz", ctypes.c_int64), ("status", ctypes.c_int32), ("checks", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class sca_batch_item(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A_dev", ctypes.c_void_p), ("lda", ctypes.c_int64), ("b_dev", ctypes.c_void_p),
                ("lambda_", ctypes.c_double), ("c", ctypes.c_double), ("beta", ctypes.c_double),
                ("tau", ctypes.c_double), ("F_star", ctypes.c_double),
                ("block_ptr_host", ctypes.POINTER(ctypes.c_int64)), ("nblocks", ctypes.c_int64),
                ("instance", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class sca_launch(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_size_t), ("grad_kind", ctypes.c_int32),
                ("grad_cols", ctypes.c_int32), ("grad_unroll", ctypes.c_int32),
                ("grad_wg_per_cu", ctypes.c_int32)]


class sca_tune_entry(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("target", ctypes.c_int32), ("m_lo", ctypes.c_int64),
                ("m_hi", ctypes.c_int64), ("launch", sca_launch)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_S = ctypes.c_int
# name -> (restype, argtypes); the declarations of include/sca.h
SIGNATURES = {
    "sca_version": (ctypes.c_char_p, []),
    "sca_last_error": (ctypes.c_char_p, []),
    "sca_problem_create_dense": (_S, [ctypes.POINTER(_P), _S, _I64, _I64, _P, _I64, _P, _D, _D,
                                      _D, ctypes.POINTER(_I64), _I64, _P]),
    "sca_problem_create_csr": (_S, [ctypes.POINTER(_P), _S, _I64, _I64, _I64, _P, _P, _P, _P,
                                    _D, _D, _D, ctypes.POINTER(_I64), _I64, _P]),
    "sca_problem_set_regularizer": (_S, [_P, _S, _D]),
    "sca_problem_update_rhs": (_S, [_P, _P, _D, _P]),
    "sca_problem_destroy": (None, [_P]),
    "sca_step": (_S, [_P, ctypes.POINTER(sca_opts), _I64, _I64, _P, _P, _P]),
    "sca_residual": (_S, [_P, _P, _P, _P]),
    "sca_select_blocks": (_S, [_P, ctypes.POINTER(sca_opts), _I64, _P, _P]),
    "sca_philox4x32_10": (_S, [_P, _P, _I64, _P]),
    "sca_objective": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(_D),
                           ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I64), _P]),
    "sca_solve": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(sca_stats), _P]),
    "sca_adjoint": (_S, [_P, ctypes.POINTER(sca_opts), _P, _P, _P, ctypes.POINTER(_D), _D, _I64,
                         _P]),
    "sca_adjoint_noalloc": (_S, [_P, ctypes.POINTER(sca_opts), _P, _P, _P, ctypes.POINTER(_D),
                                 _D, _I64, _P]),
    "sca_profile_get": (_S, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_D),
                             _S]),
    "sca_tuning_set": (_S, [ctypes.POINTER(sca_tune_entry), _I64]),
    "sca_problem_get_launch": (_S, [_P, ctypes.POINTER(sca_launch)]),
    "sca_problem_set_launch": (_S, [_P, ctypes.POINTER(sca_launch)]),
    "sca_stream_copy": (_S, [_P, _P, _I64, ctypes.c_int32, _P]),
    "sca_stream_read": (_S, [_P, _I64, _P, ctypes.c_int32, _P]),
    "sca_batch_create": (_S, [ctypes.POINTER(_P), _S, _I64, ctypes.POINTER(sca_batch_item), _P]),
    "sca_batch_destroy": (None, [_P]),
    "sca_batch_layout": (_S, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "sca_batch_get_launch": (_S, [_P, ctypes.POINTER(sca_launch)]),
    "sca_batch_set_launch": (_S, [_P, ctypes.POINTER(sca_launch)]),
    "sca_batch_set_regularizer": (_S, [_P, _S, _D]),
    "sca_batch_set_fstar": (_S, [_P, ctypes.POINTER(_D)]),
    "sca_batch_residual": (_S, [_P, _P, _P, _P]),
    "sca_batch_step": (_S, [_P, ctypes.POINTER(sca_opts), _I64, _I64, _P, _P, _P]),
    "sca_batch_solve": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(sca_stats), _P]),
    "sca_batch_update_rhs": (_S, [_P, _P, ctypes.POINTER(_D), _P]),
    "sca_batch_adjoint": (_S, [_P, ctypes.POINTER(sca_opts), _P, _P, _P, ctypes.POINTER(_D), _D,
                               _I64, _P]),
    "sca_batch_objective": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(_D),
                                 ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I64),
                                 _P]),
    "sca_multi_create": (_S, [ctypes.POINTER(_P), _S, _I64, _I64, _P, _I64, _I64, _P, _I64,
                              ctypes.POINTER(_D), _D, _D, ctypes.POINTER(_I64), _I64, _P]),
    "sca_multi_destroy": (None, [_P]),
    "sca_multi_set_fstar": (_S, [_P, ctypes.POINTER(_D)]),
    "sca_multi_residual": (_S, [_P, _P, _P, _P]),
    "sca_multi_step": (_S, [_P, ctypes.POINTER(sca_opts), _I64, _I64, _P, _P, _P]),
    "sca_multi_objective": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(_D),
                                 ctypes.POINTER(_D), ctypes.POINTER(_I64), _P]),
    "sca_multi_solve": (_S, [_P, ctypes.POINTER(sca_opts), _P, ctypes.POINTER(sca_stats), _P]),
    "sca_multi_profile_get": (_S, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), _S]),
}

_LIB = None


def lib():
    """Load libsca.so (raises when it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1701_04900_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
        load_tuning()
    return _LIB


def _check(status):
    if status != SCA_OK:
        raise SCAError(status, lib().sca_last_error().decode())
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_buf(t, name, dtype=None, numel=None):
    """The checks the C ABI cannot make: a dense (contiguous) buffer of the expected dtype
    holding at least ``numel`` elements."""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {numel} needed")


def _dptrs(*specs):
    """Device pointers of (tensor, name, dtype, numel) specs: every buffer is checked with
    _check_buf first, then each must live on the device (None passes as NULL)."""
    for sp in specs:
        _check_buf(*sp)
    out = []
    for t, name, *_ in specs:
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name}: expected a device tensor")
        out.append(None if t is None else ctypes.c_void_p(t.data_ptr()))
    return tuple(out)


def _dptr(t, name="buffer", dtype=None, numel=None):
    """Device pointer of one tensor after the checks of _check_buf."""
    return _dptrs((t, name, dtype, numel))[0]


# Shapes of the live handles created through this module (handle value -> dict), so that
# the buffers passed with a handle can be checked against its dtype and sizes before the
# call: the library sees plain pointers and cannot check their extent.
_SHAPES: dict = {}


def _shape(h):
    v = h.value if isinstance(h, ctypes.c_void_p) else h
    return _SHAPES.get(v, {})


def _forget(h):
    _SHAPES.pop(h.value if isinstance(h, ctypes.c_void_p) else h, None)


def _dtype_code(dt):
    if dt == torch.float32:
        return SCA_F32
    if dt == torch.float64:
        return SCA_F64
    raise ValueError(f"unsupported dtype {dt}")


def make_opts(gamma=0.9, tau=0.0, select_p=1.0, seed=0, instance=0, gamma_mu=0.0, flags=0,
              max_rounds=0, check_every=10, refresh_every=0, tol_rel_obj=0.0, F_star=0.0,
              tol_merit=0.0, delay_chunks=0, delay_stale=0, async_workgroups=0) -> sca_opts:
    return sca_opts(ctypes.sizeof(sca_opts), gamma, gamma_mu, tau, select_p, seed, instance,
                    flags, max_rounds, check_every, refresh_every, tol_rel_obj, F_star, tol_merit,
                    delay_chunks, delay_stale, async_workgroups)


TUNING_PATH = os.path.join(_HERE, "tuning", "gfx950.json")


def load_tuning(path=None):
    """Install the launch-shape table written by paper_1701_04900_amd.autotune (if any)."""
    import json
    path = path or os.environ.get("SCA_TUNING", TUNING_PATH)
    if not os.path.exists(path):
        return 0
    rows = json.load(open(path))["entries"]
    arr = (sca_tune_entry * len(rows))()
    for i, e in enumerate(rows):
        arr[i] = sca_tune_entry(SCA_F32 if e["dtype"] == "f32" else SCA_F64,
                                1 if e.get("target") == "batch" else 0, e["m_lo"], e["m_hi"],
                                sca_launch(ctypes.sizeof(sca_launch), e["grad_kind"],
                                           e["grad_cols"], e["grad_unroll"], e["grad_wg_per_cu"]))
    _check(_LIB.sca_tuning_set(arr, len(rows)))
    return len(rows)


def sca_tuning_set(rows):
    arr = (sca_tune_entry * len(rows))(*rows)
    _check(lib().sca_tuning_set(arr, len(rows)))


def sca_problem_get_launch(h):
    out = sca_launch()
    _check(lib().sca_problem_get_launch(h, ctypes.byref(out)))
    return dict(grad_kind=out.grad_kind, grad_cols=out.grad_cols, grad_unroll=out.grad_unroll,
                grad_wg_per_cu=out.grad_wg_per_cu)


def sca_problem_set_launch(h, grad_kind, grad_cols, grad_unroll, grad_wg_per_cu):
    l = sca_launch(ctypes.sizeof(sca_launch), grad_kind, grad_cols, grad_unroll, grad_wg_per_cu)
    _check(lib().sca_problem_set_launch(h, ctypes.byref(l)))


# ------------------------------------------------------------------ entry points
def sca_version():
    return lib().sca_version().decode()


def sca_problem_create_dense(At, m, b, lam, c, beta, block_ptr, stream=None):
    """At: (n, lda) device tensor (column-major A), b: (m,) device tensor."""
    n, lda = At.shape
    code = _dtype_code(At.dtype)
    pa, pb = _dptrs((At, "At", None, None), (b, "b", At.dtype, m))
    bp = np.ascontiguousarray(block_ptr, dtype=np.int64)
    h = ctypes.c_void_p()
    _check(lib().sca_problem_create_dense(
        ctypes.byref(h), code, m, n, pa, lda, pb, float(lam),
        float(c), float(beta), bp.ctypes.data_as(ctypes.POINTER(_I64)), len(bp) - 1,
        _stream(stream)))
    _SHAPES[h.value] = dict(dtype=At.dtype, m=m, n=n, nblocks=len(bp) - 1)
    return h


def sca_problem_create_csr(m, n, rowptr, colidx, vals, b, lam, c, beta, block_ptr, stream=None):
    code = _dtype_code(vals.dtype)
    nnz = vals.numel()
    ptrs = _dptrs((rowptr, "rowptr", torch.int64, m + 1), (colidx, "colidx", torch.int32, nnz),
                  (vals, "vals", None, None), (b, "b", vals.dtype, m))
    bp = np.ascontiguousarray(block_ptr, dtype=np.int64)
    h = ctypes.c_void_p()
    _check(lib().sca_problem_create_csr(
        ctypes.byref(h), code, m, n, nnz, *ptrs, float(lam), float(c), float(beta),
        bp.ctypes.data_as(ctypes.POINTER(_I64)), len(bp) - 1, _stream(stream)))
    _SHAPES[h.value] = dict(dtype=vals.dtype, m=m, n=n, nblocks=len(bp) - 1)
    return h


def sca_problem_set_regularizer(h, reg, theta=0.0):
    _check(lib().sca_problem_set_regularizer(h, int(reg), float(theta)))


def sca_problem_update_rhs(h, b, lam, stream=None):
    sh = _shape(h)
    pb = _dptr(b, "b", sh.get("dtype"), sh.get("m"))
    _check(lib().sca_problem_update_rhs(h, pb, float(lam), _stream(stream)))


def sca_problem_destroy(h):
    _forget(h)
    lib().sca_problem_destroy(h)


def _xr(h, x, r):
    sh = _shape(h)
    return _dptrs((x, "x", sh.get("dtype"), sh.get("n")), (r, "r", sh.get("dtype"), sh.get("m")))


def sca_step(h, opts, round_begin, nrounds, x, r, stream=None):
    px, pr = _xr(h, x, r)
    _check(lib().sca_step(h, ctypes.byref(opts), int(round_begin), int(nrounds), px, pr,
                          _stream(stream)))


def sca_residual(h, x, r, stream=None):
    px, pr = _xr(h, x, r)
    _check(lib().sca_residual(h, px, pr, _stream(stream)))


def sca_select_blocks(h, opts, k, mask, stream=None):
    pm = _dptr(mask, "mask", torch.uint8, _shape(h).get("nblocks"))
    _check(lib().sca_select_blocks(h, ctypes.byref(opts), int(k), pm, _stream(stream)))


def sca_philox4x32_10(inp, out, count, stream=None):
    _check(lib().sca_philox4x32_10(_dptr(inp), _dptr(out), int(count), _stream(stream)))


def sca_objective(h, opts, x, stream=None):
    F, mer, mf, nnz = _D(), _D(), _D(), _I64()
    sh = _shape(h)
    px = _dptr(x, "x", sh.get("dtype"), sh.get("n"))
    _check(lib().sca_objective(h, ctypes.byref(opts), px, ctypes.byref(F), ctypes.byref(mer),
                               ctypes.byref(mf), ctypes.byref(nnz), _stream(stream)))
    return dict(F=F.value, merit=mer.value, MF=mf.value, nnz=nnz.value)


def sca_solve(h, opts, x, stream=None, raise_on_notconv=True):
    st = sca_stats()
    st.struct_size = ctypes.sizeof(sca_stats)
    sh = _shape(h)
    px = _dptr(x, "x", sh.get("dtype"), sh.get("n"))
    status = lib().sca_solve(h, ctypes.byref(opts), px, ctypes.byref(st), _stream(stream))
    if status != SCA_OK and not (status == SCA_ENOTCONV and not raise_on_notconv):
        _check(status)
    return st.as_dict()


def sca_adjoint(h, opts, xstar, xbar, bbar, cg_tol=0.0, cg_maxit=0, stream=None):
    lb = _D()
    sh = _shape(h)
    dt, n, m = sh.get("dtype"), sh.get("n"), sh.get("m")
    ptrs = _dptrs((xstar, "xstar", dt, n), (xbar, "xbar", dt, n), (bbar, "bbar", dt, m))
    _check(lib().sca_adjoint(h, ctypes.byref(opts), *ptrs,
                             ctypes.byref(lb), float(cg_tol), int(cg_maxit), _stream(stream)))
    return lb.value


def sca_adjoint_noalloc(h, opts, xstar, xbar, bbar, cg_tol=0.0, cg_maxit=0, stream=None):
    lb = _D()
    sh = _shape(h)
    dt, n, m = sh.get("dtype"), sh.get("n"), sh.get("m")
    ptrs = _dptrs((xstar, "xstar", dt, n), (xbar, "xbar", dt, n), (bbar, "bbar", dt, m))
    _check(lib().sca_adjoint_noalloc(h, ctypes.byref(opts), *ptrs, ctypes.byref(lb),
                                     float(cg_tol), int(cg_maxit), _stream(stream)))
    return lb.value


def sca_profile_get(h, reset=False):
    ms = (_D * SCA_K_NKINDS)()
    n = (_I64 * SCA_K_NKINDS)()
    by = (_D * SCA_K_NKINDS)()
    _check(lib().sca_profile_get(h, ms, n, by, int(reset)))
    names = ["select", "grad", "compact", "fold"]
    return {names[k]: dict(ms=ms[k], launches=n[k], bytes=by[k]) for k in range(SCA_K_NKINDS)}


def sca_stream_copy(dst, src, nbytes, grid=0, stream=None):
    _check(lib().sca_stream_copy(_dptr(dst), _dptr(src), int(nbytes), int(grid), _stream(stream)))


def sca_stream_read(src, nbytes, sink, grid=0, stream=None):
    _check(lib().sca_stream_read(_dptr(src), int(nbytes), _dptr(sink), int(grid), _stream(stream)))


# ------------------------------------------------------------------ convenience holder
class Problem:
    """Keeps the borrowed device tensors alive for the lifetime of the library handle."""

    def __init__(self, handle, keep, m, n, dtype):
        self.handle, self._keep, self.m, self.n, self.dtype = handle, keep, m, n, dtype

    @classmethod
    def dense(cls, At, m, b, lam, c=0.0, beta=math.inf, block_ptr=None, stream=None):
        n = At.shape[0]
        if block_ptr is None:
            block_ptr = np.arange(n + 1, dtype=np.int64)
        h = sca_problem_create_dense(At, m, b, lam, c, beta, block_ptr, stream)
        return cls(h, (At, b), m, n, At.dtype)

    @classmethod
    def csr(cls, m, n, rowptr, colidx, vals, b, lam, c=0.0, beta=math.inf, block_ptr=None,
            stream=None):
        if block_ptr is None:
            block_ptr = np.arange(n + 1, dtype=np.int64)
        h = sca_problem_create_csr(m, n, rowptr, colidx, vals, b, lam, c, beta, block_ptr, stream)
        return cls(h, (b,), m, n, vals.dtype)  # the CSR may be released after create

    @classmethod
    def from_workload(cls, w, stream=None):
        if hasattr(w, "rowptr"):
            return cls.csr(w.m, w.n, w.rowptr, w.colidx, w.vals, w.b, w.lam, w.c, w.beta,
                           w.block_ptr, stream)
        return cls.dense(w.At, w.m, w.b, w.lam, w.c, w.beta, w.block_ptr, stream)

    def update_rhs(self, b, lam, stream=None):
        """Install a new right-hand side and lambda; b is borrowed, so it is kept alive here
        for as long as it is the problem's."""
        sca_problem_update_rhs(self.handle, b, lam, stream)
        self._keep = (self._keep[0], b) if len(self._keep) == 2 else (b,)

    def close(self):
        if self.handle is not None:
            sca_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batched form
def sca_batch_create(items, dtype, stream=None):
    """items: list of dicts with keys m, n, At (device (n, lda)), b (device), lam, c, beta,
    tau, F_star, block_ptr (int64 array), instance."""
    arr = (sca_batch_item * len(items))()
    keep = []
    for k, it in enumerate(items):
        _dptrs((it["At"], f"At[{k}]", dtype, None), (it["b"], f"b[{k}]", dtype, it["m"]))
        bp = np.ascontiguousarray(it["block_ptr"], dtype=np.int64)
        keep.append(bp)
        arr[k] = sca_batch_item(ctypes.sizeof(sca_batch_item), it["m"], it["n"],
                                it["At"].data_ptr(), it["At"].shape[1], it["b"].data_ptr(),
                                float(it["lam"]), float(it.get("c", 0.0)),
                                float(it.get("beta", math.inf)), float(it["tau"]),
                                float(it.get("F_star", 0.0)),
                                bp.ctypes.data_as(ctypes.POINTER(_I64)), len(bp) - 1,
                                int(it.get("instance", k)), 0)
    h = ctypes.c_void_p()
    _check(lib().sca_batch_create(ctypes.byref(h), _dtype_code(dtype), len(items), arr,
                                  _stream(stream)))
    xo, ro = sca_batch_layout(h, len(items))
    _SHAPES[h.value] = dict(dtype=dtype, K=len(items), x=int(xo[-1]), r=int(ro[-1]))
    return h


def sca_batch_destroy(h):
    _forget(h)
    lib().sca_batch_destroy(h)


def _bxr(h, x, r):
    sh = _shape(h)
    return _dptrs((x, "x_all", sh.get("dtype"), sh.get("x")),
                  (r, "r_all", sh.get("dtype"), sh.get("r")))


def sca_batch_layout(h, K):
    xo = (_I64 * (K + 1))()
    ro = (_I64 * (K + 1))()
    _check(lib().sca_batch_layout(h, xo, ro))
    return np.array(xo[:], dtype=np.int64), np.array(ro[:], dtype=np.int64)


def sca_batch_get_launch(h):
    out = sca_launch()
    _check(lib().sca_batch_get_launch(h, ctypes.byref(out)))
    return dict(grad_kind=out.grad_kind, grad_cols=out.grad_cols, grad_unroll=out.grad_unroll,
                grad_wg_per_cu=out.grad_wg_per_cu)


def sca_batch_set_launch(h, grad_kind, grad_cols=4, grad_wg_per_cu=2):
    l = sca_launch(ctypes.sizeof(sca_launch), grad_kind, grad_cols, 1, grad_wg_per_cu)
    _check(lib().sca_batch_set_launch(h, ctypes.byref(l)))


def sca_batch_set_regularizer(h, reg, theta=0.0):
    _check(lib().sca_batch_set_regularizer(h, int(reg), float(theta)))


def sca_batch_set_fstar(h, F_star):
    a = np.ascontiguousarray(F_star, dtype=np.float64)
    _check(lib().sca_batch_set_fstar(h, a.ctypes.data_as(ctypes.POINTER(_D))))


def sca_batch_residual(h, x_all, r_all, stream=None):
    _check(lib().sca_batch_residual(h, *_bxr(h, x_all, r_all), _stream(stream)))


def sca_batch_step(h, opts, round_begin, nrounds, x_all, r_all, stream=None):
    _check(lib().sca_batch_step(h, ctypes.byref(opts), int(round_begin), int(nrounds),
                                *_bxr(h, x_all, r_all), _stream(stream)))


def sca_batch_solve(h, opts, x_all, K, stream=None, raise_on_notconv=True):
    st = (sca_stats * K)()
    for k in range(K):
        st[k].struct_size = ctypes.sizeof(sca_stats)
    px = _bxr(h, x_all, None)[0]
    status = lib().sca_batch_solve(h, ctypes.byref(opts), px, st, _stream(stream))
    if status != SCA_OK and not (status == SCA_ENOTCONV and not raise_on_notconv):
        _check(status)
    return [st[k].as_dict() for k in range(K)]


def sca_batch_objective(h, opts, x_all, K, stream=None):
    F, mer, mf, nnz = (_D * K)(), (_D * K)(), (_D * K)(), (_I64 * K)()
    _check(lib().sca_batch_objective(h, ctypes.byref(opts), _bxr(h, x_all, None)[0], F, mer,
                                     mf, nnz, _stream(stream)))
    return dict(F=np.array(F[:]), merit=np.array(mer[:]), MF=np.array(mf[:]),
                nnz=np.array(nnz[:]))


def sca_batch_update_rhs(h, b_all, lam, stream=None):
    sh = _shape(h)
    a = np.ascontiguousarray(lam, dtype=np.float64)
    if "K" in sh and a.shape != (sh["K"],):
        raise ValueError(f"lam: one value per instance ({sh['K']}) expected")
    pb = _dptr(b_all, "b_all", sh.get("dtype"), sh.get("r"))
    _check(lib().sca_batch_update_rhs(h, pb, a.ctypes.data_as(ctypes.POINTER(_D)),
                                      _stream(stream)))


def sca_batch_adjoint(h, opts, xstar_all, xbar_all, bbar_all, K, cg_tol=0.0, cg_maxit=0,
                      stream=None):
    lb = (_D * K)()
    sh = _shape(h)
    dt, nx, nr = sh.get("dtype"), sh.get("x"), sh.get("r")
    ptrs = _dptrs((xstar_all, "xstar_all", dt, nx), (xbar_all, "xbar_all", dt, nx),
                  (bbar_all, "bbar_all", dt, nr))
    _check(lib().sca_batch_adjoint(h, ctypes.byref(opts), *ptrs, lb, float(cg_tol),
                                   int(cg_maxit), _stream(stream)))
    return np.array(lb[:])


class Batch:
    """Batch handle plus the per-instance device tensors it borrows."""

    def __init__(self, workloads, F_star=None, stream=None):
        self.K = len(workloads)
        self.dtype = workloads[0].dtype
        items = []
        for k, w in enumerate(workloads):
            items.append(dict(m=w.m, n=w.n, At=w.At, b=w.b, lam=w.lam, c=w.c, beta=w.beta,
                              tau=w.tau, F_star=0.0 if F_star is None else F_star[k],
                              block_ptr=w.block_ptr, instance=w.instance))
        self._keep = [(w.At, w.b) for w in workloads]
        self.handle = sca_batch_create(items, self.dtype, stream)
        self.xoff, self.roff = sca_batch_layout(self.handle, self.K)

    def close(self):
        if self.handle is not None:
            sca_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ many right-hand sides
# Layouts: At (n, lda) as for the dense problem; B (K, ldb), row k = b_k; X (K, n), row k =
# x_k; R (K, lda), row k = A x_k - b_k (rows m..lda-1 unused).
def sca_multi_create(At, m, B, lams, c=0.0, beta=math.inf, block_ptr=None, stream=None):
    n, lda = At.shape
    K, ldb = B.shape
    if block_ptr is None:
        block_ptr = np.arange(n + 1, dtype=np.int64)
    bp = np.ascontiguousarray(block_ptr, dtype=np.int64)
    la = np.ascontiguousarray(lams, dtype=np.float64)
    if la.shape != (K,):
        raise ValueError("one lambda per right-hand side")
    code = _dtype_code(At.dtype)
    pa, pB = _dptrs((At, "At", None, None), (B, "B", At.dtype, None))
    h = ctypes.c_void_p()
    _check(lib().sca_multi_create(ctypes.byref(h), code, m, n, pa, lda,
                                  K, pB, ldb, la.ctypes.data_as(ctypes.POINTER(_D)),
                                  float(c), float(beta), bp.ctypes.data_as(ctypes.POINTER(_I64)),
                                  len(bp) - 1, _stream(stream)))
    _SHAPES[h.value] = dict(dtype=At.dtype, K=K, x=K * n, r=K * lda)
    return h


def sca_multi_destroy(h):
    _forget(h)
    lib().sca_multi_destroy(h)


def sca_multi_set_fstar(h, F_star):
    a = np.ascontiguousarray(F_star, dtype=np.float64)
    _check(lib().sca_multi_set_fstar(h, a.ctypes.data_as(ctypes.POINTER(_D))))


def sca_multi_residual(h, X, R, stream=None):
    _check(lib().sca_multi_residual(h, *_bxr(h, X, R), _stream(stream)))


def sca_multi_step(h, opts, round_begin, nrounds, X, R, stream=None):
    _check(lib().sca_multi_step(h, ctypes.byref(opts), round_begin, nrounds, *_bxr(h, X, R),
                                _stream(stream)))


def sca_multi_objective(h, opts, X, K, stream=None):
    F, mer, nnz = (_D * K)(), (_D * K)(), (_I64 * K)()
    _check(lib().sca_multi_objective(h, ctypes.byref(opts), _bxr(h, X, None)[0], F, mer, nnz,
                                     _stream(stream)))
    return dict(F=np.array(F[:]), merit=np.array(mer[:]), nnz=np.array(nnz[:]))


def sca_multi_solve(h, opts, X, K, stream=None, raise_on_notconv=True):
    st = (sca_stats * K)()
    for k in range(K):
        st[k].struct_size = ctypes.sizeof(sca_stats)
    status = lib().sca_multi_solve(h, ctypes.byref(opts), _bxr(h, X, None)[0], st,
                                   _stream(stream))
    if status != SCA_OK and not (status == SCA_ENOTCONV and not raise_on_notconv):
        _check(status)
    return [st[k].as_dict() for k in range(K)]


def sca_multi_profile_get(h, reset=False):
    ms = (_D * SCA_K_NKINDS)()
    n = (_I64 * SCA_K_NKINDS)()
    _check(lib().sca_multi_profile_get(h, ms, n, int(reset)))
    names = ["select", "grad", "compact", "fold"]
    return {names[k]: dict(ms=ms[k], launches=n[k]) for k in range(SCA_K_NKINDS)}


class Multi:
    """K right-hand sides over one dense A (borrowed device tensors kept alive)."""

    def __init__(self, At, m, B, lams, c=0.0, beta=math.inf, block_ptr=None, stream=None):
        self.K, self.m, self.n = B.shape[0], m, At.shape[0]
        self.lda = At.shape[1]
        self.dtype = At.dtype
        self._keep = (At, B)
        self.handle = sca_multi_create(At, m, B, lams, c, beta, block_ptr, stream)

    def zeros_x(self):
        return torch.zeros(self.K, self.n, dtype=self.dtype, device="cuda")

    def empty_r(self):
        return torch.zeros(self.K, self.lda, dtype=self.dtype, device="cuda")

    def close(self):
        if self.handle is not None:
            sca_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ autograd
class SolveFn(torch.autograd.Function):
    """x* = argmin of the problem for right-hand side b and weight lam (forward: sca_solve
    from x = 0; backward: sca_adjoint).  ``problem`` is a Problem over the same A; its
    right-hand side and lam are replaced by the inputs."""

    @staticmethod
    def forward(ctx, b, lam, problem, opts):
        b = b.detach().contiguous()
        lam = float(lam)
        problem.update_rhs(b, lam)
        x = torch.zeros(problem.n, dtype=problem.dtype, device=b.device)
        sca_solve(problem.handle, opts, x)
        ctx.save_for_backward(x)
        ctx.problem, ctx.opts = problem, opts
        ctx.b, ctx.lam = b, lam
        return x

    @staticmethod
    def backward(ctx, xbar):
        (x,) = ctx.saved_tensors
        # the handle may have been given another (b, lam) by a later forward: the adjoint
        # takes the support and residual from the problem, so this forward's are restored
        ctx.problem.update_rhs(ctx.b, ctx.lam)
        bbar = torch.empty(ctx.problem.m, dtype=ctx.problem.dtype, device=x.device)
        lb = sca_adjoint(ctx.problem.handle, ctx.opts, x, xbar.contiguous(), bbar)
        return bbar, torch.tensor(lb, dtype=torch.float64, device=x.device), None, None


class BatchSolveFn(torch.autograd.Function):
    """The batched form of SolveFn: b_all in the batch's r layout, lam one per instance."""

    @staticmethod
    def forward(ctx, b_all, lam, batch, opts):
        b_all = b_all.detach().contiguous()
        lam_host = lam.detach().double().cpu().numpy().copy()
        sca_batch_update_rhs(batch.handle, b_all, lam_host)
        x = torch.zeros(int(batch.xoff[-1]), dtype=batch.dtype, device=b_all.device)
        sca_batch_solve(batch.handle, opts, x, batch.K)
        ctx.save_for_backward(x)
        ctx.batch, ctx.opts = batch, opts
        ctx.b_all, ctx.lam, ctx.lam_device = b_all, lam_host, lam.device
        return x

    @staticmethod
    def backward(ctx, xbar):
        (x,) = ctx.saved_tensors
        # restore this forward's right-hand sides and weights (a later forward may have
        # replaced them; the batch copies b, so the saved tensor is what is re-installed)
        sca_batch_update_rhs(ctx.batch.handle, ctx.b_all, ctx.lam)
        bbar = torch.zeros(int(ctx.batch.roff[-1]), dtype=ctx.batch.dtype, device=x.device)
        lb = sca_batch_adjoint(ctx.batch.handle, ctx.opts, x, xbar.contiguous(), bbar,
                               ctx.batch.K)
        return bbar, torch.as_tensor(lb, dtype=torch.float64, device=ctx.lam_device), None, None
