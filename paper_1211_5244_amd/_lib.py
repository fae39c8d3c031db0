"""ctypes binding of libpoisson's C ABI (include/poisson.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  There is no fallback; if the library is missing, loading it raises.
Function names and arguments mirror the C entry points.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpoisson.so")

POISSON_OK = 0
POISSON_E_ARG = -1
POISSON_E_UNSUPPORTED = -2
POISSON_E_NO_KERNEL = -3
POISSON_E_NOMEM = -4
POISSON_E_HIP = -5
POISSON_E_STATE = -6

POISSON_FREE_X, POISSON_FREE_Y, POISSON_FREE_Z = 1, 2, 4
POISSON_FP32, POISSON_SPLIT_FP16, POISSON_SPLIT_BF16 = 0, 1, 2

# every symbol include/poisson.h declares
EXPORTED = (
    "poisson_plan", "poisson_plan_ordered", "poisson_plan_describe",
    "poisson_plan_describe_ordered", "poisson_plan_info", "poisson_plan_rows", "poisson_set_workspace",
    "poisson_kernel_set", "poisson_kernel_build", "poisson_kernel_build_isf", "poisson_kernel_get",
    "poisson_solve",
    "poisson_solve_passes", "poisson_solve_host", "poisson_solve_host_many",
    "poisson_plan_destroy", "poisson_batch_create", "poisson_batch_kernel_build",
    "poisson_batch_kernel_build_isf",
    "poisson_batch_solve", "poisson_batch_destroy", "poisson_plan_set_schedule",
    "poisson_batch_set_schedule", "poisson_batch_get_schedule", "poisson_plan_get_schedule",
    "poisson_plan_tune", "poisson_set_tune_cache", "poisson_batch_tune", "poisson_batch_set_streams",
    "poisson_batch_get_streams", "poisson_batch_set_mode", "poisson_batch_get_mode",
    "poisson_queue_radices", "poisson_batch_set_queue_radix", "poisson_batch_get_queue_radix",
    "poisson_batch_set_queue_shape", "poisson_batch_set_queue_spin", "poisson_batch_queue_status",
    "poisson_queue_simulate", "poisson_rel_l2", "poisson_rel_l2_noalloc",
    "poisson_last_error",
)

# batch modes (poisson_batch_set_mode)
POISSON_BATCH_GROUPED, POISSON_BATCH_QUEUE = 0, 1
QUEUE_ERR_SPIN = 1  # poisson_batch_queue_status: a bounded wait ran out

# schedules per pass (poisson_plan_set_schedule): tile width in bits 0-1,
# XCD-blocked workgroup order in bit 2, small-grid plane kernel in bit 3 (of
# pass 2 only)
TILE_SCHEDULES = 16
PLANE_BIT = 8


class PoissonError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i = ctypes.c_int
_u = ctypes.c_uint
_d = ctypes.c_double
_sz = ctypes.c_size_t


def load_library(path=None):
    """Load libpoisson.so (built in-tree by paper_1211_5244_amd.build)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1211_5244_amd.build`")
    lib = ctypes.CDLL(p)
    sig = {
        "poisson_plan": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _u, _d, _i]),
        "poisson_plan_describe": (_i, [_i, _i, _i, _u, _i, ctypes.POINTER(_i), ctypes.POINTER(_i),
                                       ctypes.POINTER(_sz), ctypes.POINTER(_d)]),
        "poisson_plan_rows": (_i, [_i, _i, _i, _u, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_i)]),
        "poisson_plan_ordered": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _u, _d, _i, ctypes.POINTER(_i)]),
        "poisson_plan_describe_ordered": (_i, [_i, _i, _i, _u, _i, ctypes.POINTER(_i), ctypes.POINTER(_i),
                                               ctypes.POINTER(_i), ctypes.POINTER(_sz), ctypes.POINTER(_d),
                                               ctypes.POINTER(ctypes.c_longlong)]),
        "poisson_plan_info": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_sz),
                                   ctypes.POINTER(_d)]),
        "poisson_set_workspace": (_i, [_vp, _vp, _sz]),
        "poisson_kernel_set": (_i, [_vp, _vp, _i]),
        "poisson_kernel_build": (_i, [_vp, _vp]),
        "poisson_kernel_build_isf": (_i, [_vp, _i, _vp]),
        "poisson_kernel_get": (_i, [_vp, _vp]),
        "poisson_solve": (_i, [_vp, _vp, _vp, _vp]),
        "poisson_solve_passes": (_i, [_vp, _vp, _vp, _i, _i, _vp]),
        "poisson_solve_host": (_i, [_vp, _vp, _vp, _vp]),
        "poisson_solve_host_many": (_i, [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
        "poisson_plan_destroy": (_i, [_vp]),
        "poisson_batch_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_i), ctypes.POINTER(_u),
                                      ctypes.POINTER(_d), _i]),
        "poisson_batch_kernel_build": (_i, [_vp, _vp]),
        "poisson_batch_solve": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
        "poisson_batch_destroy": (_i, [_vp]),
        "poisson_plan_set_schedule": (_i, [_vp, ctypes.POINTER(_i)]),
        "poisson_batch_set_schedule": (_i, [_vp, ctypes.POINTER(_i)]),
        "poisson_batch_get_schedule": (_i, [_vp, _i, ctypes.POINTER(_i)]),
        "poisson_plan_get_schedule": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "poisson_plan_tune": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d), _vp]),
        "poisson_batch_tune": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i,
                                    ctypes.POINTER(_d), _vp]),
        "poisson_set_tune_cache": (_i, [ctypes.c_char_p]),
        "poisson_batch_kernel_build_isf": (_i, [_vp, _i, _vp]),
        "poisson_batch_set_streams": (_i, [_vp, _i]),
        "poisson_batch_get_streams": (_i, [_vp, ctypes.POINTER(_i)]),
        "poisson_batch_set_mode": (_i, [_vp, _i]),
        "poisson_batch_get_mode": (_i, [_vp, ctypes.POINTER(_i)]),
        "poisson_queue_radices": (_i, [_i, _i, ctypes.POINTER(_i)]),
        "poisson_batch_set_queue_radix": (_i, [_vp, _i, _i]),
        "poisson_batch_get_queue_radix": (_i, [_vp, _i, ctypes.POINTER(_i)]),
        "poisson_batch_set_queue_shape": (_i, [_vp, _i, _i]),
        "poisson_batch_set_queue_spin": (_i, [_vp, _u]),
        "poisson_batch_queue_status": (_i, [_vp, ctypes.POINTER(_u)]),
        "poisson_queue_simulate": (_i, [_i, ctypes.POINTER(_i), _i, _i, _u,
                                        ctypes.POINTER(ctypes.c_longlong)]),
        "poisson_rel_l2": (_i, [_vp, _vp, _sz, ctypes.POINTER(_d), _vp]),
        "poisson_rel_l2_noalloc": (_i, [_vp, _vp, _sz, _vp, _vp]),
        "poisson_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def poisson_last_error():
    return load_library().poisson_last_error().decode()


def _check(rc):
    if rc != POISSON_OK:
        raise PoissonError(rc, poisson_last_error())


def _ptr(x):
    """Device/host address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot take the address of {type(x).__name__}")


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream on ROCm wraps a hipStream_t


def poisson_plan(n1, n2, n3, bc_mask, h, precision=POISSON_FP32):
    out = _vp()
    _check(load_library().poisson_plan(ctypes.byref(out), n1, n2, n3, bc_mask, h, precision))
    return out.value


def poisson_plan_ordered(n1, n2, n3, bc_mask, h, precision=POISSON_FP32, axis_order=None):
    out = _vp()
    order = None if axis_order is None else (_i * 3)(*[int(a) for a in axis_order])
    _check(load_library().poisson_plan_ordered(ctypes.byref(out), n1, n2, n3, bc_mask, h, precision,
                                               order))
    return out.value


def poisson_plan_describe_ordered(n1, n2, n3, bc_mask, precision=POISSON_FP32, axis_order=None):
    force = None if axis_order is None else (_i * 3)(*[int(a) for a in axis_order])
    order = (_i * 3)()
    S = (_i * 3)()
    ws = _sz()
    alg = _d()
    rows = (ctypes.c_longlong * 3)()
    _check(load_library().poisson_plan_describe_ordered(n1, n2, n3, bc_mask, precision, force, order, S,
                                                        ctypes.byref(ws), ctypes.byref(alg), rows))
    return dict(axis_order=tuple(order), S=tuple(S), workspace_bytes=ws.value, alg_bytes=alg.value,
                rows=tuple(rows))


def poisson_plan_info(plan):
    order = (_i * 3)()
    S = (_i * 3)()
    ws = _sz()
    alg = _d()
    _check(load_library().poisson_plan_info(plan, order, S, ctypes.byref(ws), ctypes.byref(alg)))
    return dict(axis_order=tuple(order), S=tuple(S), workspace_bytes=ws.value, alg_bytes=alg.value)


def poisson_plan_describe(n1, n2, n3, bc_mask, precision=POISSON_FP32):
    order = (_i * 3)()
    S = (_i * 3)()
    ws = _sz()
    alg = _d()
    _check(load_library().poisson_plan_describe(n1, n2, n3, bc_mask, precision, order, S,
                                                ctypes.byref(ws), ctypes.byref(alg)))
    return dict(axis_order=tuple(order), S=tuple(S), workspace_bytes=ws.value, alg_bytes=alg.value)


def poisson_plan_rows(n1, n2, n3, bc_mask):
    rows = (ctypes.c_longlong * 3)()
    lens = (_i * 3)()
    _check(load_library().poisson_plan_rows(n1, n2, n3, bc_mask, rows, lens))
    return tuple(rows), tuple(lens)


def poisson_set_workspace(plan, dev_ptr, nbytes):
    _check(load_library().poisson_set_workspace(plan, _ptr(dev_ptr), nbytes))


def poisson_kernel_set(plan, kf_octant, is_device_ptr=None):
    """kf_octant: float64 octant as a numpy array (host) or a device tensor."""
    if isinstance(kf_octant, np.ndarray):
        arr = np.ascontiguousarray(kf_octant, dtype=np.float64)
        _check(load_library().poisson_kernel_set(plan, arr.ctypes.data, 0))
        return
    dev = 1 if is_device_ptr is None else int(is_device_ptr)
    _check(load_library().poisson_kernel_set(plan, _ptr(kf_octant), dev))


def poisson_kernel_build(plan, stream=None):
    _check(load_library().poisson_kernel_build(plan, _stream(stream)))


def poisson_kernel_build_isf(plan, order=16, stream=None):
    _check(load_library().poisson_kernel_build_isf(plan, int(order), _stream(stream)))


def poisson_kernel_get(plan, S):
    out = np.empty((S[2] // 2 + 1, S[1] // 2 + 1, S[0] // 2 + 1), dtype=np.float64)
    _check(load_library().poisson_kernel_get(plan, out.ctypes.data))
    return out


def poisson_solve(plan, rho, V, stream=None):
    _check(load_library().poisson_solve(plan, _ptr(rho), _ptr(V), _stream(stream)))


def poisson_solve_passes(plan, rho, V, first, last, stream=None):
    _check(load_library().poisson_solve_passes(plan, _ptr(rho), _ptr(V), first, last, _stream(stream)))


def poisson_solve_host(plan, rho_host, V_host, stream=None):
    """rho_host / V_host: host addresses (pinned torch CPU tensors or ints)."""
    _check(load_library().poisson_solve_host(plan, _ptr(rho_host), _ptr(V_host), _stream(stream)))


def poisson_solve_host_many(plan, rho_list, V_list, stream=None):
    count = len(rho_list)
    r = (_vp * count)(*[_ptr(x) for x in rho_list])
    v = (_vp * count)(*[_ptr(x) for x in V_list])
    _check(load_library().poisson_solve_host_many(plan, count, r, v, _stream(stream)))


def poisson_plan_destroy(plan):
    _check(load_library().poisson_plan_destroy(plan))


def poisson_batch_create(n_list, bc_list, h_list, precision=POISSON_FP32):
    count = len(n_list)
    n = (_i * (3 * count))(*[int(v) for nn in n_list for v in nn])
    bc = (_u * count)(*[int(b) for b in bc_list])
    h = (_d * count)(*[float(x) for x in h_list])
    out = _vp()
    _check(load_library().poisson_batch_create(ctypes.byref(out), count, n, bc, h, precision))
    return out.value


def poisson_batch_kernel_build(batch, stream=None):
    _check(load_library().poisson_batch_kernel_build(batch, _stream(stream)))


def poisson_batch_solve(batch, rho_list, V_list, stream=None):
    count = len(rho_list)
    r = (_vp * count)(*[_ptr(x) for x in rho_list])
    v = (_vp * count)(*[_ptr(x) for x in V_list])
    _check(load_library().poisson_batch_solve(batch, r, v, _stream(stream)))


def poisson_batch_destroy(batch):
    _check(load_library().poisson_batch_destroy(batch))


def poisson_rel_l2(v, ref, count, stream=None):
    out = _d()
    _check(load_library().poisson_rel_l2(_ptr(v), _ptr(ref), count, ctypes.byref(out), _stream(stream)))
    return out.value


def poisson_rel_l2_noalloc(v, ref, count, out_dev, stream=None):
    """Enqueues the residual; the float64 result lands in device memory
    out_dev (a tensor or an address)."""
    _check(load_library().poisson_rel_l2_noalloc(_ptr(v), _ptr(ref), count, _ptr(out_dev),
                                                 _stream(stream)))


def poisson_plan_set_schedule(plan, tile_sel):
    arr = (_i * 5)(*[int(x) for x in tile_sel])
    _check(load_library().poisson_plan_set_schedule(plan, arr))


def poisson_batch_set_schedule(batch, tile_sel):
    arr = (_i * 5)(*[int(x) for x in tile_sel])
    _check(load_library().poisson_batch_set_schedule(batch, arr))


def poisson_batch_get_schedule(batch, index):
    sel = (_i * 5)()
    _check(load_library().poisson_batch_get_schedule(batch, int(index), sel))
    return tuple(sel)


def poisson_plan_get_schedule(plan):
    """(tile_sel[5], tile_lines[5])"""
    sel = (_i * 5)()
    lines = (_i * 5)()
    _check(load_library().poisson_plan_get_schedule(plan, sel, lines))
    return tuple(sel), tuple(lines)


def poisson_plan_tune(plan, rho, V, reps=0, stream=None):
    """Returns the chosen schedule's time per pass in ms."""
    ms = (_d * 5)()
    _check(load_library().poisson_plan_tune(plan, _ptr(rho), _ptr(V), int(reps), ms, _stream(stream)))
    return tuple(ms)


def poisson_batch_kernel_build_isf(batch, order=16, stream=None):
    _check(load_library().poisson_batch_kernel_build_isf(batch, int(order), _stream(stream)))


def poisson_set_tune_cache(path):
    """Tuned-schedule cache file (None switches it off)."""
    _check(load_library().poisson_set_tune_cache(None if path is None else str(path).encode()))


def poisson_batch_set_streams(batch, streams):
    _check(load_library().poisson_batch_set_streams(batch, int(streams)))


def poisson_batch_get_streams(batch):
    out = _i()
    _check(load_library().poisson_batch_get_streams(batch, ctypes.byref(out)))
    return out.value


def poisson_batch_tune(batch, rho_list, V_list, reps=0, stream=None):
    """Returns the chosen intermediates budget per launch in MiB."""
    count = len(rho_list)
    r = (_vp * count)(*[_ptr(x) for x in rho_list])
    v = (_vp * count)(*[_ptr(x) for x in V_list])
    mb = _d()
    _check(load_library().poisson_batch_tune(batch, r, v, int(reps), ctypes.byref(mb), _stream(stream)))
    return mb.value


def poisson_batch_set_mode(batch, mode):
    _check(load_library().poisson_batch_set_mode(batch, int(mode)))


def poisson_batch_get_mode(batch):
    out = _i()
    _check(load_library().poisson_batch_get_mode(batch, ctypes.byref(out)))
    return out.value


def poisson_queue_radices(length, radix_sel):
    """Radices of a queue transform of this length, first stage first."""
    rad = (_i * 12)()
    n = load_library().poisson_queue_radices(int(length), int(radix_sel), rad)
    _check(min(n, 0))
    return tuple(rad[:n])


def poisson_batch_set_queue_radix(batch, length, radix_sel):
    _check(load_library().poisson_batch_set_queue_radix(batch, int(length), int(radix_sel)))


def poisson_batch_get_queue_radix(batch, length):
    out = _i()
    _check(load_library().poisson_batch_get_queue_radix(batch, int(length), ctypes.byref(out)))
    return out.value


def poisson_batch_set_queue_shape(batch, tile_elems, item_kb):
    _check(load_library().poisson_batch_set_queue_shape(batch, int(tile_elems), int(item_kb)))


def poisson_batch_set_queue_spin(batch, spin_limit):
    _check(load_library().poisson_batch_set_queue_spin(batch, int(spin_limit)))


def poisson_batch_queue_status(batch):
    """Waits for the device; returns and clears the sticky queue flags."""
    out = _u()
    _check(load_library().poisson_batch_queue_status(batch, ctypes.byref(out)))
    return out.value


def poisson_queue_simulate(seg_items, workers, fault=0, seed=1):
    """Host simulation of the queue protocol; seg_items[pass][solve] items per
    segment.  Returns (waits, releases, violations, waits that ran out)."""
    nsolve = len(seg_items[0])
    flat = (_i * (5 * nsolve))(*[int(seg_items[k][i]) for k in range(5) for i in range(nsolve)])
    stats = (ctypes.c_longlong * 4)()
    _check(load_library().poisson_queue_simulate(nsolve, flat, int(workers), int(fault), int(seed), stats))
    return tuple(stats)
