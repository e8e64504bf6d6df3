"""ctypes binding of libdgtns (include/dgtns.h): the same names, argument
marshalling only.  Every computation runs in the HIP library."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgtns.so")

DGTNS_OK = 0
DGTNS_EINVAL = 1
DGTNS_ELATTICE = 2
DGTNS_ENOTFRAME = 3
DGTNS_EUNSUPPORTED = 4
DGTNS_EDEVICE = 5
DGTNS_EWORKSPACE = 6
DGTNS_ESTATE = 7

DGTNS_C64 = 0
DGTNS_C128 = 1

DGTNS_SEPARABLE = 0
DGTNS_TIME_SHEAR = 1
DGTNS_FREQ_SHEAR = 2
DGTNS_MULTIWINDOW = 3
DGTNS_FIR = 4
DGTNS_SHEAR_OLA = 5

DGTNS_ALG_SHEAR = 0
DGTNS_ALG_MULTIWINDOW = 1
DGTNS_ALG_FIR = 2
DGTNS_ALG_SHEAR_OLA = 3
DGTNS_ALG_AUTO = 4

DGTNS_OP_FORWARD = 0
DGTNS_OP_ADJOINT = 1
DGTNS_OP_WINDOW_GRAD = 2
DGTNS_OP_SET_WINDOW = 3
DGTNS_OP_DUAL = 4

c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p


class dgtns_plan_info_t(ctypes.Structure):
    _fields_ = [
        ("L", c_i64), ("a", c_i64), ("M", c_i64), ("lambda1", c_i64), ("lambda2", c_i64),
        ("b", c_i64), ("N", c_i64), ("s", c_i64), ("s0", c_i64), ("s1", c_i64), ("b_r", c_i64),
        ("branch", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("inner_a", c_i64), ("inner_M", c_i64), ("c", c_i64), ("d", c_i64), ("p", c_i64), ("q", c_i64),
        ("max_batch", c_i64), ("persistent_bytes", ctypes.c_size_t), ("windows", c_i64),
        ("block", c_i64), ("block_dgt_length", c_i64), ("real_row", c_i64),
    ]


class DgtnsError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


STATUS_NAMES = {
    0: "DGTNS_OK", 1: "DGTNS_EINVAL", 2: "DGTNS_ELATTICE", 3: "DGTNS_ENOTFRAME",
    4: "DGTNS_EUNSUPPORTED", 5: "DGTNS_EDEVICE", 6: "DGTNS_EWORKSPACE", 7: "DGTNS_ESTATE",
}

# (name, restype, argtypes) for every symbol of include/dgtns.h
SIGNATURES = [
    ("dgtns_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("dgtns_last_error", ctypes.c_char_p, []),
    ("dgtns_plan_create", ctypes.c_int, [ctypes.POINTER(c_vp), c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.c_int, c_i64]),
    ("dgtns_plan_create_alg", ctypes.c_int,
     [ctypes.POINTER(c_vp), c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.c_int, c_i64, ctypes.c_int]),
    ("dgtns_plan_create_fir", ctypes.c_int,
     [ctypes.POINTER(c_vp), c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.c_int, c_i64, c_i64, c_i64]),
    ("dgtns_plan_create_ola", ctypes.c_int,
     [ctypes.POINTER(c_vp), c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.c_int, c_i64, c_i64, c_i64, c_i64]),
    ("dgtns_plan_create_ola_alg", ctypes.c_int,
     [ctypes.POINTER(c_vp), c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.c_int, c_i64, c_i64, c_i64, c_i64,
      ctypes.c_int]),
    ("dgtns_plan_info", ctypes.c_int, [c_vp, ctypes.POINTER(dgtns_plan_info_t)]),
    ("dgtns_plan_bind", ctypes.c_int, [c_vp, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_workspace_bytes", ctypes.c_int, [c_vp, ctypes.c_int, c_i64, ctypes.POINTER(ctypes.c_size_t)]),
    ("dgtns_set_window", ctypes.c_int, [c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_forward", ctypes.c_int, [c_vp, c_vp, ctypes.c_int, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_forward_real", ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_adjoint_real", ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_forward_noalloc", ctypes.c_int, [c_vp, c_vp, ctypes.c_int, c_vp, c_i64, c_vp]),
    ("dgtns_forward_batch", ctypes.c_int, [c_vp, ctypes.POINTER(c_vp), ctypes.c_int, ctypes.POINTER(c_vp), c_i64,
                                           c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_adjoint", ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_window_grad", ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_dual_window", ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_tight_window", ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    ("dgtns_check_op", ctypes.c_int, [c_vp, ctypes.c_int, c_i64]),
    ("dgtns_plan_destroy", ctypes.c_int, [c_vp]),
    ("dgtns_shearfind", ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_i64, ctypes.POINTER(c_i64)]),
    ("dgtns_noshear_factor", ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, ctypes.POINTER(c_i64)]),
    ("dgtns_timing_enable", ctypes.c_int, [ctypes.c_int]),
    ("dgtns_timing_collect", ctypes.c_int, []),
    ("dgtns_timing_entry", ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(c_i64),
                                          ctypes.POINTER(ctypes.c_double)]),
    ("dgtns_timing_reset", ctypes.c_int, []),
]

_lib = None


def lib():
    """Load libdgtns.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1307_4569_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def check(status: int, where: str):
    if status != DGTNS_OK:
        raise DgtnsError(status, where, lib().dgtns_last_error().decode())


def _call(name, *args):
    check(getattr(lib(), name)(*args), name)


def dgtns_plan_create(L, a, M, lambda1, lambda2, dtype, max_batch):
    h = c_vp()
    _call("dgtns_plan_create", ctypes.byref(h), L, a, M, lambda1, lambda2, dtype, max_batch)
    return h


def dgtns_plan_create_alg(L, a, M, lambda1, lambda2, dtype, max_batch, algorithm):
    h = c_vp()
    _call("dgtns_plan_create_alg", ctypes.byref(h), L, a, M, lambda1, lambda2, dtype, max_batch, algorithm)
    return h


def dgtns_plan_create_fir(L, a, M, lambda1, lambda2, dtype, max_batch, g_start, g_len):
    h = c_vp()
    _call("dgtns_plan_create_fir", ctypes.byref(h), L, a, M, lambda1, lambda2, dtype, max_batch, g_start, g_len)
    return h


def dgtns_plan_create_ola(L, a, M, lambda1, lambda2, dtype, max_batch, g_start, g_len, block):
    h = c_vp()
    _call("dgtns_plan_create_ola", ctypes.byref(h), L, a, M, lambda1, lambda2, dtype, max_batch, g_start, g_len,
          block)
    return h


def dgtns_plan_create_ola_alg(L, a, M, lambda1, lambda2, dtype, max_batch, g_start, g_len, block, inner_algorithm):
    h = c_vp()
    _call("dgtns_plan_create_ola_alg", ctypes.byref(h), L, a, M, lambda1, lambda2, dtype, max_batch, g_start,
          g_len, block, inner_algorithm)
    return h


def dgtns_plan_info(plan):
    info = dgtns_plan_info_t()
    _call("dgtns_plan_info", plan, ctypes.byref(info))
    return info


def dgtns_plan_bind(plan, dev_ptr, nbytes, stream):
    _call("dgtns_plan_bind", plan, dev_ptr, nbytes, stream)


def dgtns_workspace_bytes(plan, op, B):
    n = ctypes.c_size_t()
    _call("dgtns_workspace_bytes", plan, op, B, ctypes.byref(n))
    return n.value


def dgtns_set_window(plan, g_ptr, ws_ptr, ws_bytes, stream):
    _call("dgtns_set_window", plan, g_ptr, ws_ptr, ws_bytes, stream)


def dgtns_forward(plan, f_ptr, real_input, c_ptr, B, ws_ptr, ws_bytes, stream):
    _call("dgtns_forward", plan, f_ptr, int(real_input), c_ptr, B, ws_ptr, ws_bytes, stream)


def dgtns_forward_real(plan, f_ptr, c_ptr, B, ws_ptr, ws_bytes, stream):
    _call("dgtns_forward_real", plan, f_ptr, c_ptr, B, ws_ptr, ws_bytes, stream)


def dgtns_adjoint_real(plan, c_ptr, f_ptr, B, ws_ptr, ws_bytes, stream):
    _call("dgtns_adjoint_real", plan, c_ptr, f_ptr, B, ws_ptr, ws_bytes, stream)


DGTNS_NOALLOC_SCRATCH_BYTES = 64 << 20


def dgtns_forward_noalloc(plan, f_ptr, real_input, c_ptr, B, stream):
    _call("dgtns_forward_noalloc", plan, f_ptr, int(real_input), c_ptr, B, stream)


DGTNS_MAX_LIST_BATCH = 16


def dgtns_forward_batch(plan, f_ptrs, real_input, c_ptrs, ws_ptr, ws_bytes, stream):
    B = len(f_ptrs)
    fa = (c_vp * B)(*f_ptrs)
    ca = (c_vp * B)(*c_ptrs)
    _call("dgtns_forward_batch", plan, fa, int(real_input), ca, B, ws_ptr, ws_bytes, stream)


def dgtns_adjoint(plan, c_ptr, f_ptr, B, ws_ptr, ws_bytes, stream):
    _call("dgtns_adjoint", plan, c_ptr, f_ptr, B, ws_ptr, ws_bytes, stream)


def dgtns_window_grad(plan, f_ptr, gc_ptr, gg_ptr, B, ws_ptr, ws_bytes, stream):
    _call("dgtns_window_grad", plan, f_ptr, gc_ptr, gg_ptr, B, ws_ptr, ws_bytes, stream)


def dgtns_dual_window(plan, g_ptr, gd_ptr, bounds_ptr, ws_ptr, ws_bytes, stream):
    _call("dgtns_dual_window", plan, g_ptr, gd_ptr, bounds_ptr, ws_ptr, ws_bytes, stream)


def dgtns_tight_window(plan, g_ptr, gt_ptr, bounds_ptr, ws_ptr, ws_bytes, stream):
    _call("dgtns_tight_window", plan, g_ptr, gt_ptr, bounds_ptr, ws_ptr, ws_bytes, stream)


def dgtns_check_op(plan, op, B):
    _call("dgtns_check_op", plan, op, B)


def dgtns_plan_destroy(plan):
    _call("dgtns_plan_destroy", plan)


def dgtns_shearfind(L, a, M, lambda1, lambda2):
    out = (c_i64 * 3)()
    _call("dgtns_shearfind", L, a, M, lambda1, lambda2, out)
    return int(out[0]), int(out[1]), int(out[2])


def dgtns_noshear_factor(a, M, lambda1, lambda2):
    out = c_i64()
    _call("dgtns_noshear_factor", a, M, lambda1, lambda2, ctypes.byref(out))
    return int(out.value)


def dgtns_timing_enable(on):
    _call("dgtns_timing_enable", int(on))


def dgtns_timing_collect():
    n = lib().dgtns_timing_collect()
    if n < 0 or n > 1000:
        check(n, "dgtns_timing_collect")
    return n


def dgtns_timing_entry(i):
    name = ctypes.create_string_buffer(128)
    cnt = c_i64()
    ms = ctypes.c_double()
    _call("dgtns_timing_entry", i, name, 128, ctypes.byref(cnt), ctypes.byref(ms))
    return name.value.decode(), int(cnt.value), float(ms.value)


def dgtns_timing_reset():
    _call("dgtns_timing_reset")


def kernel_times():
    """{kernel name: (launches, total ms)} of the launches timed since the
    last reset."""
    n = dgtns_timing_collect()
    return {name: (cnt, ms) for name, cnt, ms in (dgtns_timing_entry(i) for i in range(n))}


def dgtns_status_string(status):
    return lib().dgtns_status_string(status).decode()


def dgtns_last_error():
    return lib().dgtns_last_error().decode()
