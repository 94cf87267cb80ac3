"""ctypes binding of libtsk (include/tsk.h).  Argument marshalling only: every
step of the computation runs in the HIP library; torch supplies device memory
and the current HIP stream."""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsk.so")

MAX_ORDER = 8
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENUMERIC = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
DENSE, COO = 0, 1
SKETCH = {"ts": 0, "lev": 1, "lev_det": 2}
INIT = {"rrf": 0, "random": 1, "user": 2}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
SOLVE = {"exact": 0, "rsvd": 1}
FLAG_RECORD_FIT = 1
FLAG_FINAL_FIT = 2


class TskError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tsk status {status}: {msg}")
        self.status = status


class _Tensor(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_ORDER),
                ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("values", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("idx", ctypes.c_void_p * MAX_ORDER)]


class _Options(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_int32), ("m", ctypes.c_int64), ("init", ctypes.c_int32),
                ("rrf_k1", ctypes.c_int32), ("rrf_k2", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("flags", ctypes.c_uint32), ("solve", ctypes.c_int32),
                ("rsvd_k", ctypes.c_int32), ("first_sweep", ctypes.c_int32),
                ("tol", ctypes.c_double)]


_lib = None


def lib():
    """Load libtsk.so; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run paper_2104_01101_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sz = ctypes.POINTER(ctypes.c_size_t)
        T, O = ctypes.POINTER(_Tensor), ctypes.POINTER(_Options)
        sig = {
            "tsk_abi_version": (i32, []),
            "tsk_last_error": (ctypes.c_char_p, []),
            "tsk_stream_key": (u64, [u64, i32, i64, i64, i64]),
            "tsk_draw": (u64, [u64, u64]),
            "tsk_workspace_size": (i32, [T, vp, O, sz]),
            "tsk_tucker_sketch_als": (i32, [T, vp, O, vp, vp, vp, vp]),
            "tsk_cp_workspace_size": (i32, [T, i32, vp, O, sz]),
            "tsk_cp_via_tucker": (i32, [T, i32, vp, i32, O, vp, vp]),
            "tsk_hash_tables": (i32, [i32, vp, i32, i64, u64, vp, vp, vp]),
            "tsk_sketch_rhs_ts": (i32, [T, i32, i64, vp, vp, vp, vp, sz, vp]),
            "tsk_sketch_lhs_ts": (i32, [i32, vp, vp, i32, i64, vp, vp, vp, i32, vp, vp, sz, vp]),
            "tsk_rc_solve": (i32, [vp, vp, i64, i64, i64, i32, i32, vp, vp, vp, sz, vp]),
            "tsk_rsvd_solve": (i32, [vp, vp, i64, i64, i64, i32, i32, vp, i32, vp, vp, vp, sz,
                                     vp]),
            "tsk_rsvd_solve_noalloc": (i32, [vp, vp, i64, i64, i64, i32, i32, vp, i32, vp, vp,
                                             vp]),
            "tsk_rrf_init": (i32, [T, i32, i32, i32, i32, u64, vp, vp, sz, vp]),
            "tsk_leverage_sample": (i32, [i32, vp, vp, i32, i64, u64, i32, vp, vp, vp, vp, sz, vp]),
            "tsk_leverage_select": (i32, [i32, vp, vp, i32, i64, vp, vp, vp, sz, vp]),
            "tsk_sketch_lev": (i32, [T, vp, i32, i64, vp, vp, vp, i32, vp, vp, vp]),
            "tsk_fiber_index": (i32, [T, i32, vp, sz, vp, sz, vp]),
            "tsk_sketch_lev_coo": (i32, [T, i32, vp, i64, vp, vp, i32, vp, vp]),
            "tsk_fit": (i32, [T, vp, vp, vp, vp, vp, sz, vp]),
            "tsk_sketched_residual_fwd": (i32, [i32, vp, vp, i32, i64, vp, vp, vp, vp, vp, i32,
                                                vp, vp, sz, vp]),
            "tsk_sketched_residual_bwd": (i32, [i32, vp, vp, i32, i64, vp, vp, vp, vp, vp, i32,
                                                vp, vp, vp, sz, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != OK:
        raise TskError(status, lib().tsk_last_error().decode())


# ---------------------------------------------------------------- helpers ----
def stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def ptr_array(ts, ctype=ctypes.c_void_p):
    arr = (ctype * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr() if t is not None else 0
    return arr


def i64_array(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def i32_array(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def workspace(nbytes, device):
    """Device byte buffer aligned to 256 bytes; returns (keepalive, pointer)."""
    buf = torch.empty(int(nbytes) + 512, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    aligned = (base + 255) & ~255
    return buf, ctypes.c_void_p(aligned), int(nbytes)


def query_and_alloc(fn, args_before, args_after, device):
    """Run fn(*args_before, ws, &bytes, *args_after) with a workspace query first."""
    nb = ctypes.c_size_t(0)
    check(fn(*args_before, None, ctypes.byref(nb), *args_after))
    keep, wp, n = workspace(nb.value, device)
    nb2 = ctypes.c_size_t(n)
    check(fn(*args_before, wp, ctypes.byref(nb2), *args_after))
    return keep
