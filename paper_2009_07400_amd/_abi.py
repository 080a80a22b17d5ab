"""ctypes binding of the C ABI in include/tmd.h (argument marshalling only).

Every function here has the name of the C entry point it calls and raises
TmdError when the call returns a status other than TMD_OK.  Pointers are
plain integers (device addresses), streams are hipStream_t handles as
integers (0 = default stream).  Nothing in this module computes.
"""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtinymd_amd.so")

TMD_OK = 0
TMD_EINVAL = -1
TMD_EBOX = -2
TMD_ESTATE = -3
TMD_ENBR_OVERFLOW = -4
TMD_ENONFINITE = -5
TMD_EWORKSPACE = -6
TMD_EHIP = -7

TIMING_CLASSES = ("force", "neighbor", "binning", "drift", "thermo", "copy", "adjoint")

TMD_MODEL_LJ = 0
TMD_MODEL_SPRING_DASHPOT = 1


class TmdParams(C.Structure):
    _fields_ = [
        ("epsilon", C.c_double),
        ("sigma", C.c_double),
        ("mass", C.c_double),
        ("cutoff", C.c_double),
        ("skin", C.c_double),
        ("dt", C.c_double),
        ("rebuild_every", C.c_int32),
        ("max_neighbors", C.c_int32),
        ("stiffness", C.c_double),
        ("damping", C.c_double),
        ("model", C.c_int32),
        ("reserved", C.c_int32),
    ]


class TmdInfo(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int64),
        ("n_padded", C.c_int64),
        ("cells_per_axis", C.c_int32),
        ("max_neighbors", C.c_int32),
        ("n_cells", C.c_int64),
        ("workspace_bytes", C.c_size_t),
        ("step", C.c_int64),
        ("n_boxes", C.c_int32),
        ("n_blocks", C.c_int32),
        ("block_threads", C.c_int32),
        ("lds_atoms", C.c_int32),
        ("block_edge", C.c_int32),
        ("block_parts", C.c_int32),
        ("lanes_per_atom", C.c_int32),
        ("build_threads", C.c_int32),
        ("build_lanes", C.c_int32),
        ("graph_captures", C.c_int32),
        ("graph_launches", C.c_int64),
        ("half_list", C.c_int32),
        ("layout", C.c_int32),
    ]


class TmdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None
_P = C.c_void_p
_S = C.c_int


def load_library():
    """Load libtinymd_amd.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python paper_2009_07400_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "tmd_create": (_S, [C.POINTER(TmdParams), C.c_int64, C.c_double, C.POINTER(_P)]),
        "tmd_create_batch": (_S, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(TmdParams),
                                  C.POINTER(_P)]),
        "tmd_workspace_size": (_S, [_P, C.POINTER(C.c_size_t)]),
        "tmd_bind_workspace": (_S, [_P, _P, C.c_size_t]),
        "tmd_set_state": (_S, [_P, _P, _P, C.c_int64, _P]),
        "tmd_build_neighbors": (_S, [_P, _P]),
        "tmd_compute_forces": (_S, [_P, _P, _P, _P]),
        "tmd_integrate": (_S, [_P, C.c_int32, C.c_int32, _P, _P]),
        "tmd_get_state": (_S, [_P, _P, _P, C.POINTER(C.c_int64), _P]),
        "tmd_get_neighbors": (_S, [_P, _P, _P, C.c_int64, _P]),
        "tmd_sync": (_S, [_P, _P]),
        "tmd_get_info": (_S, [_P, C.POINTER(TmdInfo)]),
        "tmd_set_schedule": (_S, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "tmd_set_half_list": (_S, [_P, C.c_int32]),
        "tmd_set_layout": (_S, [_P, C.c_int32, _P]),
        "tmd_set_lj_params": (_S, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double), _P]),
        "tmd_adjoint_workspace_size": (_S, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
        "tmd_adjoint_forward": (_S, [_P, C.c_int32, _P, C.c_size_t, _P]),
        "tmd_adjoint_backward": (_S, [_P, _P, C.c_size_t, _P, _P, _P, _P, _P, _P, _P]),
        "tmd_autotune": (_S, [_P, C.c_int32, C.c_int32, _P]),
        "tmd_set_timing": (_S, [_P, C.c_int32]),
        "tmd_set_graphs": (_S, [_P, C.c_int32]),
        "tmd_get_timing": (_S, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "tmd_compute_forces_static": (_S, [C.POINTER(TmdParams), C.c_int64, C.c_double, _P, _P, _P, _P, _P]),
        "tmd_status_string": (C.c_char_p, [_S]),
        "tmd_last_error": (C.c_char_p, [_P]),
        "tmd_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, handle=None):
    if st != TMD_OK:
        lib = load_library()
        msg = lib.tmd_status_string(st).decode()
        if handle:
            detail = lib.tmd_last_error(handle).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise TmdError(st, msg)


def _p3(ptrs):
    if ptrs is None:
        return None
    arr = (_P * 3)(*[p if p else None for p in ptrs])
    return arr


def tmd_status_string(status: int) -> str:
    return load_library().tmd_status_string(status).decode()


def tmd_last_error(handle) -> str:
    return load_library().tmd_last_error(handle).decode()


def tmd_create(params: TmdParams, n_atoms: int, box_length: float):
    h = _P()
    _check(load_library().tmd_create(C.byref(params), n_atoms, box_length, C.byref(h)))
    return h


def tmd_create_batch(params, n_atoms, box_lengths):
    """params: one TmdParams per box."""
    nb = len(n_atoms)
    if len(params) != nb or len(box_lengths) != nb:
        raise ValueError("one TmdParams, atom count and box length per box")
    h = _P()
    _check(load_library().tmd_create_batch(nb, (C.c_int64 * nb)(*n_atoms), (C.c_double * nb)(*box_lengths),
                                           (TmdParams * nb)(*params), C.byref(h)))
    return h


def tmd_workspace_size(handle) -> int:
    n = C.c_size_t()
    _check(load_library().tmd_workspace_size(handle, C.byref(n)), handle)
    return int(n.value)


def tmd_bind_workspace(handle, dev_ptr: int, nbytes: int) -> None:
    _check(load_library().tmd_bind_workspace(handle, dev_ptr, nbytes), handle)


def tmd_set_state(handle, pos_ptrs, vel_ptrs, step: int, stream: int) -> None:
    p, v = _p3(pos_ptrs), _p3(vel_ptrs)
    _check(load_library().tmd_set_state(handle, C.cast(p, _P) if p is not None else None,
                                         C.cast(v, _P) if v is not None else None, step, stream), handle)


def tmd_build_neighbors(handle, stream: int) -> None:
    _check(load_library().tmd_build_neighbors(handle, stream), handle)


def tmd_compute_forces(handle, f_ptrs, energy_virial_ptr, stream: int) -> None:
    f = _p3(f_ptrs)
    _check(load_library().tmd_compute_forces(handle, C.cast(f, _P) if f is not None else None,
                                              energy_virial_ptr, stream), handle)


def tmd_compute_forces_static(params: TmdParams, n_atoms: int, box_length: float, pos_ptrs, f_ptrs,
                              energy_virial_ptr, status_ptr, stream: int) -> None:
    p, f = _p3(pos_ptrs), _p3(f_ptrs)
    _check(load_library().tmd_compute_forces_static(C.byref(params), n_atoms, box_length,
                                                     C.cast(p, _P) if p is not None else None,
                                                     C.cast(f, _P) if f is not None else None,
                                                     energy_virial_ptr, status_ptr, stream))


def tmd_integrate(handle, n_steps: int, thermo_every: int, thermo_ptr, stream: int) -> None:
    _check(load_library().tmd_integrate(handle, n_steps, thermo_every, thermo_ptr, stream), handle)


def tmd_get_state(handle, pos_ptrs, vel_ptrs, stream: int) -> int:
    step = C.c_int64()
    p, v = _p3(pos_ptrs), _p3(vel_ptrs)
    _check(load_library().tmd_get_state(handle, C.cast(p, _P) if p is not None else None,
                                         C.cast(v, _P) if v is not None else None, C.byref(step), stream), handle)
    return int(step.value)


def tmd_get_neighbors(handle, counts_ptr: int, ids_ptr: int, capacity: int, stream: int) -> None:
    _check(load_library().tmd_get_neighbors(handle, counts_ptr, ids_ptr, capacity, stream), handle)


def tmd_sync(handle, stream: int) -> None:
    _check(load_library().tmd_sync(handle, stream), handle)


def tmd_get_info(handle) -> dict:
    info = TmdInfo()
    _check(load_library().tmd_get_info(handle, C.byref(info)), handle)
    return {k: getattr(info, k) for k, _ in TmdInfo._fields_}


def tmd_set_schedule(handle, threads: int, lds_atoms: int, block_edge: int = 0, block_parts: int = 0,
                     lanes_per_atom: int = 0, build_threads: int = 0, build_lanes: int = 0) -> None:
    _check(load_library().tmd_set_schedule(handle, threads, lds_atoms, block_edge, block_parts, lanes_per_atom,
                                           build_threads, build_lanes),
           handle)


TMD_LAYOUT_SOA, TMD_LAYOUT_AOS, TMD_LAYOUT_AOSOA = 0, 1, 2


def tmd_set_layout(handle, layout: int, stream: int) -> None:
    _check(load_library().tmd_set_layout(handle, layout, stream), handle)


def tmd_set_half_list(handle, half: int) -> None:
    _check(load_library().tmd_set_half_list(handle, half), handle)


def tmd_set_lj_params(handle, epsilon, sigma, stream: int) -> None:
    nb = len(epsilon)
    _check(load_library().tmd_set_lj_params(handle, (C.c_double * nb)(*epsilon), (C.c_double * nb)(*sigma),
                                             stream), handle)


def tmd_adjoint_workspace_size(handle, n_steps: int) -> int:
    n = C.c_size_t()
    _check(load_library().tmd_adjoint_workspace_size(handle, n_steps, C.byref(n)), handle)
    return int(n.value)


def tmd_adjoint_forward(handle, n_steps: int, ws_ptr: int, nbytes: int, stream: int) -> None:
    _check(load_library().tmd_adjoint_forward(handle, n_steps, ws_ptr, nbytes, stream), handle)


def tmd_adjoint_backward(handle, ws_ptr: int, nbytes: int, lam_x, lam_v, grad_x0, grad_v0, grad_eps_ptr,
                         grad_sigma_ptr, stream: int) -> None:
    arrs = [_p3(a) for a in (lam_x, lam_v, grad_x0, grad_v0)]
    ptrs = [C.cast(a, _P) if a is not None else None for a in arrs]
    _check(load_library().tmd_adjoint_backward(handle, ws_ptr, nbytes, *ptrs, grad_eps_ptr, grad_sigma_ptr, stream),
           handle)


TMD_TUNE_ADJOINT = 1


def tmd_autotune(handle, repeats: int, stream: int, flags: int = 0) -> None:
    _check(load_library().tmd_autotune(handle, repeats, flags, stream), handle)


def tmd_set_timing(handle, enable: bool) -> None:
    _check(load_library().tmd_set_timing(handle, 1 if enable else 0), handle)


def tmd_set_graphs(handle, enable: bool) -> None:
    _check(load_library().tmd_set_graphs(handle, 1 if enable else 0), handle)


def tmd_get_timing(handle) -> dict:
    ms = (C.c_double * len(TIMING_CLASSES))()
    n = (C.c_int64 * len(TIMING_CLASSES))()
    _check(load_library().tmd_get_timing(handle, ms, n), handle)
    return {name: (float(ms[k]), int(n[k])) for k, name in enumerate(TIMING_CLASSES)}


def tmd_destroy(handle) -> None:
    if handle:
        load_library().tmd_destroy(handle)
