"""ctypes binding of the C ABI in include/selinv.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors (or raw device addresses) handed over as plain
pointers; streams are raw hipStream_t handles.  No arithmetic of the method
happens in Python.
"""

from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libselinv.so")

SELINV_R64, SELINV_C128, SELINV_H128, SELINV_LU64 = 0, 1, 2, 3
SCHED_PERSISTENT, SCHED_LEVELS, SCHED_PUSH = 0, 1, 2
STATUS = {0: "OK", 1: "EINVAL", 2: "EPATTERN", 3: "ESINGULAR", 4: "ENOMEM", 5: "EDEVICE", 6: "ESTATE",
          7: "EUNSUPPORTED"}

EXPORTED = (
    "selinv_default_opts", "selinv_version", "selinv_tune_key", "selinv_analyze", "selinv_symbolic", "selinv_sizes",
    "selinv_factor", "selinv_normalize", "selinv_factor_host", "selinv_factor_device", "selinv_run", "selinv_normalize_run", "selinv_normalize_run_noalloc", "selinv_extract",
    "selinv_scatter",
    "selinv_backward",
    "selinv_logdet", "selinv_check_plan", "selinv_trace", "selinv_items", "selinv_sync", "selinv_last_error", "selinv_error_info", "selinv_destroy",
)


class Opts(C.Structure):
    _fields_ = [("max_super", C.c_int32), ("dtype", C.c_int32), ("batch", C.c_int32), ("sched", C.c_int32),
                ("relax", C.c_double), ("nthreads", C.c_int32), ("dense_min_c", C.c_int32),
                ("watchdog_ms", C.c_int64), ("dense_max_bytes", C.c_int64), ("split_min_k", C.c_int32),
                ("adjoint", C.c_int32), ("tune_cache", C.c_char_p)]


_P64 = C.POINTER(C.c_int64)
_P32 = C.POINTER(C.c_int32)


class SymbolicView(C.Structure):
    _fields_ = [("n", C.c_int64), ("nsuper", C.c_int64), ("nnzL", C.c_int64), ("panel_elems", C.c_int64),
                ("batch", C.c_int64), ("dtype", C.c_int64),
                ("perm", _P64), ("parent", _P64), ("colcount", _P64), ("xsuper", _P64), ("sparent", _P64),
                ("rowptr", _P64), ("rowind_L", _P64), ("panel_off", _P64),
                ("seg_ptr", _P64), ("seg_super", _P64), ("seg_start", _P64), ("seg_posoff", _P64),
                ("posarr", _P32), ("nseg", C.c_int64), ("nposarr", C.c_int64),
                ("flops_exact", C.c_double), ("flops", C.c_double), ("depth", C.c_int64),
                ("tuned_nodes", C.c_int64)]


class Sizes(C.Structure):
    _fields_ = [("panels_bytes", C.c_int64), ("x_bytes", C.c_int64), ("work_bytes", C.c_int64),
                ("dtilde_bytes", C.c_int64), ("abar_bytes", C.c_int64), ("trace_bytes", C.c_int64),
                ("tables_bytes", C.c_int64)]


class SelinvError(RuntimeError):
    def __init__(self, status, msg, info0=-1, info1=-1):
        super().__init__(f"selinv {STATUS.get(status, status)}: {msg} (info {info0}, {info1})")
        self.status = status
        self.info = (info0, info1)


_lib = None


def load():
    """Load the shared library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "selinv_default_opts": (None, [C.POINTER(Opts)]),
        "selinv_version": (C.c_char_p, []),
        "selinv_tune_key": (C.c_char_p, []),
        "selinv_analyze": (C.c_int, [C.c_int64, vp, vp, vp, C.POINTER(Opts), C.POINTER(vp)]),
        "selinv_symbolic": (C.c_int, [vp, C.POINTER(SymbolicView)]),
        "selinv_sizes": (C.c_int, [vp, C.POINTER(Sizes)]),
        "selinv_factor": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "selinv_normalize": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "selinv_factor_host": (C.c_int, [vp, vp, vp]),
        "selinv_factor_device": (C.c_int, [vp, vp, vp, vp, vp]),
        "selinv_run": (C.c_int, [vp, vp, vp, vp, vp]),
        "selinv_normalize_run": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "selinv_normalize_run_noalloc": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "selinv_extract": (C.c_int, [vp, vp, vp, vp, vp]),
        "selinv_scatter": (C.c_int, [vp, vp, vp, vp, vp]),
        "selinv_backward": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "selinv_logdet": (C.c_int, [vp, vp]),
        "selinv_check_plan": (C.c_int, [vp]),
        "selinv_trace": (C.c_int, [vp, vp]),
        "selinv_items": (C.c_int, [vp, C.c_int32, C.POINTER(_P32), C.POINTER(C.c_int64)]),
        "selinv_sync": (C.c_int, [vp, vp]),
        "selinv_last_error": (C.c_char_p, [vp]),
        "selinv_error_info": (C.c_int64, [vp, C.c_int]),
        "selinv_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(ctx, status):
    if status != 0:
        lib = load()
        msg = lib.selinv_last_error(ctx).decode() if ctx else "no context"
        raise SelinvError(status, msg, lib.selinv_error_info(ctx, 0) if ctx else -1,
                          lib.selinv_error_info(ctx, 1) if ctx else -1)


def ptr(x):
    """Address of a numpy array, a torch tensor or an int; None -> NULL."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return x.ctypes.data


# --- one wrapper per C entry point -------------------------------------------

def selinv_default_opts():
    o = Opts()
    load().selinv_default_opts(C.byref(o))
    return o


def selinv_version():
    return load().selinv_version().decode()


def selinv_tune_key():
    return load().selinv_tune_key().decode()


def selinv_analyze(n, colptr, rowind, perm, opts):
    lib = load()
    h = C.c_void_p()
    st = lib.selinv_analyze(n, ptr(colptr), ptr(rowind), ptr(perm), C.byref(opts), C.byref(h))
    if st != 0:
        err = SelinvError(st, lib.selinv_last_error(h).decode() if h.value else "analyze failed",
                          lib.selinv_error_info(h, 0) if h.value else -1,
                          lib.selinv_error_info(h, 1) if h.value else -1)
        if h.value:
            lib.selinv_destroy(h)
        raise err
    return h


def selinv_symbolic(h):
    v = SymbolicView()
    check(h, load().selinv_symbolic(h, C.byref(v)))
    return v


def selinv_sizes(h):
    s = Sizes()
    check(h, load().selinv_sizes(h, C.byref(s)))
    return s


def selinv_factor(h, values, panels, work, dtilde, stream):
    check(h, load().selinv_factor(h, ptr(values), ptr(panels), ptr(work), ptr(dtilde), stream))


def selinv_normalize(h, ldlt, panels, work, dtilde, stream):
    check(h, load().selinv_normalize(h, ptr(ldlt), ptr(panels), ptr(work), ptr(dtilde), stream))


def selinv_factor_host(h, values, panels_host):
    check(h, load().selinv_factor_host(h, ptr(values), ptr(panels_host)))


def selinv_factor_device(h, values, ldlt, work, stream):
    check(h, load().selinv_factor_device(h, ptr(values), ptr(ldlt), ptr(work), stream))


def selinv_run(h, panels, x, work, stream):
    check(h, load().selinv_run(h, ptr(panels), ptr(x), ptr(work), stream))


def selinv_normalize_run(h, ldlt, panels, x, work, dtilde, stream):
    check(h, load().selinv_normalize_run(h, ptr(ldlt), ptr(panels), ptr(x), ptr(work), ptr(dtilde), stream))


def selinv_normalize_run_noalloc(h, ldlt, panels, x, dtilde, stream):
    check(h, load().selinv_normalize_run_noalloc(h, ptr(ldlt), ptr(panels), ptr(x), ptr(dtilde), stream))


def selinv_extract(h, x, work, out, stream):
    check(h, load().selinv_extract(h, ptr(x), ptr(work), ptr(out), stream))


def selinv_scatter(h, vals, work, panel, stream):
    check(h, load().selinv_scatter(h, ptr(vals), ptr(work), ptr(panel), stream))


def selinv_backward(h, panels, x, dtilde, xbar, wlogdet, work, abar, stream):
    check(h, load().selinv_backward(h, ptr(panels), ptr(x), ptr(dtilde), ptr(xbar), ptr(wlogdet), ptr(work),
                                    ptr(abar), stream))


def selinv_logdet(h, out_host):
    check(h, load().selinv_logdet(h, ptr(out_host)))


def selinv_check_plan(h):
    check(h, load().selinv_check_plan(h))


def selinv_trace(h, trace):
    check(h, load().selinv_trace(h, ptr(trace)))


def selinv_items(h, which=0):
    """Host copy of the work items, int32 [n, 4] rows {K, type, a, b}
    (which = 0: the forward traversal, 1: the adjoint in launch order, 2: the
    forward level launches {kind, items per matrix, first item type, depth},
    3: the normalization chunks {first level launch, depth, entries, 0},
    4: the subtree group ranges {group, level launch, first, end})."""
    import numpy as np

    p = _P32()
    n = C.c_int64()
    check(h, load().selinv_items(h, which, C.byref(p), C.byref(n)))
    return np.ctypeslib.as_array(p, shape=(n.value, 4)).copy() if n.value else np.zeros((0, 4), np.int32)


def selinv_sync(h, stream):
    check(h, load().selinv_sync(h, stream))


def selinv_last_error(h):
    return load().selinv_last_error(h).decode()


def selinv_error_info(h, which):
    return load().selinv_error_info(h, which)


def selinv_destroy(h):
    load().selinv_destroy(h)
