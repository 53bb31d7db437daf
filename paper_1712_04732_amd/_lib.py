"""ctypes binding of libse_mi355x.so with the names of include/se.h.

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libse_mi355x.so")

# se_status
SE_OK = 0
SE_ERR_ARG = 1
SE_ERR_PARAM = 2
SE_ERR_NONNEUTRAL = 3
SE_ERR_OUT_OF_BOX = 4
SE_ERR_NONFINITE = 5
SE_ERR_DEVICE = 6
SE_ERR_NOMEM = 7
SE_ERR_UNSUPPORTED = 8
SE_ERR_WORKSPACE = 9

SE_WIN_GAUSSIAN = 0
SE_WIN_PKB = 1
SE_WIN_ES = 2
SE_F64 = 0
SE_F32 = 1

SE_IN_F32 = 0x1
SE_ADD_SELF = 0x2
SE_SYNC_CHECK = 0x4
SE_OUT_GRAD = 0x8
SE_ALLOW_NONNEUTRAL = 0x10
SE_PROFILE = 0x20
SE_ACCUMULATE = 0x40


class se_params(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int),
        ("L", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("M", ctypes.c_int),
        ("P", ctypes.c_int),
        ("window", ctypes.c_int),
        ("shape", ctypes.c_double),
        ("nu", ctypes.c_int),
        ("lambda_", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("s", ctypes.c_double),
        ("n_l", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("Q", ctypes.c_double),
        ("prec", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("tile3", ctypes.c_int * 3),
        ("fft_cap", ctypes.c_int),
        ("xcd_tiles", ctypes.c_int),
        ("xcd_fft", ctypes.c_int),
        ("spread_mode", ctypes.c_int),
        ("force_method", ctypes.c_int),
        ("deriv_fit", ctypes.c_int),
        ("My", ctypes.c_int),
        ("Mz", ctypes.c_int),
    ]


class se_tune_report(ctypes.Structure):
    _fields_ = [
        ("candidates", ctypes.c_int),
        ("ms_default", ctypes.c_double),
        ("ms_tuned", ctypes.c_double),
    ]


class se_plan_info(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int),
        ("M", ctypes.c_int),
        ("P", ctypes.c_int),
        ("nu", ctypes.c_int),
        ("Mt", ctypes.c_int),
        ("n0", ctypes.c_int),
        ("nI", ctypes.c_int),
        ("n_l", ctypes.c_int),
        ("grid", ctypes.c_int * 3),
        ("nfft", ctypes.c_int * 3),
        ("tile", ctypes.c_int * 3),
        ("fft_cap", ctypes.c_int),
        ("spread_mode", ctypes.c_int),
        ("fft_wide", ctypes.c_int),
        ("h", ctypes.c_double),
        ("shape", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("s", ctypes.c_double),
        ("R", ctypes.c_double),
        ("device_bytes", ctypes.c_size_t),
        ("workspace_bytes", ctypes.c_size_t),
        ("fft_block", ctypes.c_int * 5),
    ]


class se_stage_record(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_int),
        ("ms_total", ctypes.c_double),
        ("bytes", ctypes.c_double),
        ("flops", ctypes.c_double),
    ]


class SEError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {se_status_string(status)} (status {status})")


_lib = None

_SIGS = {
    "se_params_default": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.POINTER(se_params)]),
    "se_plan_create": (ctypes.c_int, [ctypes.POINTER(se_params), ctypes.c_long, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "se_plan_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(se_plan_info)]),
    "se_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint,
                               ctypes.c_void_p]),
    "se_eval_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint,
                                      ctypes.c_void_p]),
    "se_get_device_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "se_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "se_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "se_plan_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(se_stage_record),
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "se_params_for_tolerance": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(se_params)]),
    "se_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(se_params), ctypes.POINTER(ctypes.c_long), ctypes.c_int,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "se_batch_plan_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(se_plan_info),
                                              ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int)]),
    "se_eval_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint, ctypes.c_void_p]),
    "se_batch_plan_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(se_stage_record),
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "se_batch_get_device_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "se_batch_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "se_autotune": (ctypes.c_int, [ctypes.POINTER(se_params), ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_uint, ctypes.c_void_p, ctypes.POINTER(se_params),
                                   ctypes.POINTER(se_tune_report)]),
    "se_rs_cells": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_long, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "se_rs_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "se_rs_cells_box": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_long, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "se_rs_plan_create_box": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                             ctypes.c_double,
                                             ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "se_rs_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "se_rs_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint,
                                  ctypes.c_void_p]),
    "se_rs_get_device_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "se_rs_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "se_rs_plan_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(se_stage_record),
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "se_error_scale": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]),
    "se_rs_cutoff_for_tolerance": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "se_params_recipe": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(se_params)]),
    "se_plan_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "se_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "se_batch_plan_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "se_batch_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "se_rs_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "se_rs_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "se_eval_vjp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_uint, ctypes.c_void_p]),
    "se_energy_vjp": (ctypes.c_int, [ctypes.c_long, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_uint, ctypes.c_void_p]),
    "se_batch_autotune": (ctypes.c_int, [ctypes.POINTER(se_params), ctypes.POINTER(ctypes.c_long), ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint, ctypes.c_void_p,
                                         ctypes.POINTER(se_params), ctypes.POINTER(se_tune_report)]),
}


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with python -m paper_1712_04732_amd.build_lib")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def se_status_string(status: int) -> str:
    return load().se_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != SE_OK:
        raise SEError(status, what)


def se_params_default(D, L, xi, M, P, window, Q, tol, prec):
    out = se_params()
    _check(load().se_params_default(int(D), float(L), float(xi), int(M), int(P), int(window),
                                    float(Q), float(tol), int(prec), ctypes.byref(out)),
           "se_params_default")
    return out


def se_plan_create(params: se_params, n_max: int, stream: int = 0) -> ctypes.c_void_p:
    plan = ctypes.c_void_p()
    _check(load().se_plan_create(ctypes.byref(params), int(n_max), ctypes.c_void_p(stream),
                                 ctypes.byref(plan)), "se_plan_create")
    return plan


def se_plan_get_info(plan) -> se_plan_info:
    info = se_plan_info()
    _check(load().se_plan_get_info(plan, ctypes.byref(info)), "se_plan_get_info")
    return info


def _ws_size(fn, plan, what):
    b = ctypes.c_size_t()
    _check(fn(plan, ctypes.byref(b)), what)
    return b.value


def se_plan_workspace_size(plan) -> int:
    return _ws_size(load().se_plan_workspace_size, plan, "se_plan_workspace_size")


def se_plan_set_workspace(plan, ptr, nbytes):
    _check(load().se_plan_set_workspace(plan, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)),
           "se_plan_set_workspace")


def se_batch_plan_workspace_size(plan) -> int:
    return _ws_size(load().se_batch_plan_workspace_size, plan, "se_batch_plan_workspace_size")


def se_batch_plan_set_workspace(plan, ptr, nbytes):
    _check(load().se_batch_plan_set_workspace(plan, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)),
           "se_batch_plan_set_workspace")


def se_rs_workspace_size(plan) -> int:
    return _ws_size(load().se_rs_workspace_size, plan, "se_rs_workspace_size")


def se_rs_set_workspace(plan, ptr, nbytes):
    _check(load().se_rs_set_workspace(plan, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)), "se_rs_set_workspace")


def se_eval_vjp(plan, N, xyz_ptr, q_ptr, g_ptr, grad_phi_ptr, grad_x_ptr, grad_q_ptr, flags, stream) -> int:
    """Returns the status (callers decide whether to raise)."""
    return load().se_eval_vjp(plan, int(N), ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr), ctypes.c_void_p(g_ptr),
                              ctypes.c_void_p(grad_phi_ptr), ctypes.c_void_p(grad_x_ptr),
                              ctypes.c_void_p(grad_q_ptr), ctypes.c_uint(flags), ctypes.c_void_p(stream))


def se_energy_vjp(N, prec, grad_E_ptr, q_ptr, phi_ptr, grad_phi_ptr, grad_x_ptr, grad_q_ptr, flags, stream) -> int:
    """Returns the status (callers decide whether to raise)."""
    return load().se_energy_vjp(int(N), int(prec), ctypes.c_void_p(grad_E_ptr), ctypes.c_void_p(q_ptr),
                                ctypes.c_void_p(phi_ptr), ctypes.c_void_p(grad_phi_ptr), ctypes.c_void_p(grad_x_ptr),
                                ctypes.c_void_p(grad_q_ptr), ctypes.c_uint(flags), ctypes.c_void_p(stream))


def se_eval(plan, N, xyz_ptr, q_ptr, phi_ptr, force_ptr, energy_ptr, flags, stream) -> int:
    """Returns the status (callers decide whether to raise)."""
    return load().se_eval(plan, int(N), ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr),
                          ctypes.c_void_p(phi_ptr), ctypes.c_void_p(force_ptr),
                          ctypes.c_void_p(energy_ptr), ctypes.c_uint(flags), ctypes.c_void_p(stream))


SE_STATIC_SCRATCH_BYTES = 128 << 20


def se_eval_static(plan, N, xyz_ptr, q_ptr, phi_ptr, force_ptr, energy_ptr, flags, stream) -> int:
    """se_eval with the library's static scratch as workspace (allocates
    nothing).  Returns the status (callers decide whether to raise)."""
    return load().se_eval_static(plan, int(N), ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr),
                                 ctypes.c_void_p(phi_ptr), ctypes.c_void_p(force_ptr),
                                 ctypes.c_void_p(energy_ptr), ctypes.c_uint(flags), ctypes.c_void_p(stream))


def se_get_device_status(plan, stream) -> int:
    return load().se_get_device_status(plan, ctypes.c_void_p(stream))


def se_plan_profile(plan, stream, reset=True):
    """List of dicts {name, launches, ms_total, ms_avg, bytes, flops} per launch site."""
    cap = 64
    arr = (se_stage_record * cap)()
    n = ctypes.c_int()
    _check(load().se_plan_profile(plan, ctypes.c_void_p(stream), arr, cap, ctypes.byref(n), int(reset)),
           "se_plan_profile")
    out = []
    for i in range(n.value):
        r = arr[i]
        out.append(dict(name=r.name.decode(), launches=r.launches, ms_total=r.ms_total,
                        ms_avg=r.ms_total / max(r.launches, 1), bytes=r.bytes, flops=r.flops))
    return out


def se_params_for_tolerance(D, L, xi, Q, tol_rel, P, window, prec):
    out = se_params()
    _check(load().se_params_for_tolerance(int(D), float(L), float(xi), float(Q), float(tol_rel), int(P),
                                          int(window), int(prec), ctypes.byref(out)), "se_params_for_tolerance")
    return out


def se_params_recipe(D, L, xi, Q, tol_rel, window, prec):
    """Section 6: M and P from the tolerance (with the error-pollution remedy)."""
    out = se_params()
    _check(load().se_params_recipe(int(D), float(L), float(xi), float(Q), float(tol_rel), int(window), int(prec),
                                   ctypes.byref(out)), "se_params_recipe")
    return out


def se_error_scale(Q, xi, L):
    """B of Section 5.2 (relative tolerances are rms tolerances over B)."""
    b = ctypes.c_double()
    _check(load().se_error_scale(float(Q), float(xi), float(L), ctypes.byref(b)), "se_error_scale")
    return b.value


def se_rs_cutoff_for_tolerance(L, xi, Q, tol_rel):
    """Real-space cutoff of Eq. (KP_rc) for the relative tolerance tol_rel."""
    rc = ctypes.c_double()
    _check(load().se_rs_cutoff_for_tolerance(float(L), float(xi), float(Q), float(tol_rel), ctypes.byref(rc)),
           "se_rs_cutoff_for_tolerance")
    return rc.value


def se_batch_plan_create(params, N, stream=0):
    n = len(params)
    arr = (se_params * n)(*params)
    narr = (ctypes.c_long * n)(*[int(v) for v in N])
    plan = ctypes.c_void_p()
    _check(load().se_batch_plan_create(arr, narr, n, ctypes.c_void_p(stream), ctypes.byref(plan)),
           "se_batch_plan_create")
    return plan


def se_batch_plan_get_info(plan, sys):
    info = se_plan_info()
    n = ctypes.c_long()
    blocks = ctypes.c_int()
    _check(load().se_batch_plan_get_info(plan, int(sys), ctypes.byref(info), ctypes.byref(n), ctypes.byref(blocks)),
           "se_batch_plan_get_info")
    return info, n.value, blocks.value


def se_eval_batch(plan, xyz_ptr, q_ptr, phi_ptr, force_ptr, energy_ptr, flags, stream) -> int:
    return load().se_eval_batch(plan, ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr), ctypes.c_void_p(phi_ptr),
                                ctypes.c_void_p(force_ptr), ctypes.c_void_p(energy_ptr), ctypes.c_uint(flags),
                                ctypes.c_void_p(stream))


def se_batch_plan_profile(plan, stream, reset=True):
    """List of dicts per stage launch, then the whole evaluation
    ("batch_all_stages"), as for se_plan_profile."""
    cap = 32
    arr = (se_stage_record * cap)()
    n = ctypes.c_int()
    _check(load().se_batch_plan_profile(plan, ctypes.c_void_p(stream), arr, cap, ctypes.byref(n), int(reset)),
           "se_batch_plan_profile")
    out = []
    for i in range(n.value):
        r = arr[i]
        out.append(dict(name=r.name.decode(), launches=r.launches, ms_total=r.ms_total,
                        ms_avg=r.ms_total / max(r.launches, 1), bytes=r.bytes, flops=r.flops))
    return out


def se_autotune(params, N, xyz_ptr, q_ptr, flags, stream):
    """Tuned copy of params and the report (dict)."""
    out = se_params()
    rep = se_tune_report()
    _check(load().se_autotune(ctypes.byref(params), int(N), ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr),
                              int(flags), ctypes.c_void_p(stream), ctypes.byref(out), ctypes.byref(rep)),
           "se_autotune")
    return out, dict(candidates=rep.candidates, ms_default=rep.ms_default, ms_tuned=rep.ms_tuned)


def se_batch_autotune(params, N, xyz_ptr, q_ptr, flags, stream):
    n = len(params)
    arr = (se_params * n)(*params)
    outs = (se_params * n)()
    Ns = (ctypes.c_long * n)(*[int(v) for v in N])
    rep = se_tune_report()
    _check(load().se_batch_autotune(arr, Ns, n, ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr), int(flags),
                                    ctypes.c_void_p(stream), outs, ctypes.byref(rep)), "se_batch_autotune")
    return [outs[i] for i in range(n)], dict(candidates=rep.candidates, ms_default=rep.ms_default,
                                             ms_tuned=rep.ms_tuned)


def se_rs_cells(L, rc, n_max, cells_per_rc=0):
    """(cells per direction, neighbour span) of the real-space cell list."""
    c, sp = ctypes.c_int(), ctypes.c_int()
    _check(load().se_rs_cells(float(L), float(rc), int(n_max), int(cells_per_rc), ctypes.byref(c), ctypes.byref(sp)),
           "se_rs_cells")
    return c.value, sp.value


def se_rs_plan_create(D, L, xi, rc, n_max, prec, cells_per_rc=0, stream=0):
    plan = ctypes.c_void_p()
    _check(load().se_rs_plan_create(int(D), float(L), float(xi), float(rc), int(n_max), int(prec),
                                    int(cells_per_rc), ctypes.c_void_p(stream), ctypes.byref(plan)),
           "se_rs_plan_create")
    return plan


def se_rs_cells_box(Ls, rc, n_max, cells_per_rc=0):
    """(cells, spans) per direction of the real-space cell list in a
    rectangular box of sides Ls."""
    sides = (ctypes.c_double * 3)(*[float(v) for v in Ls])
    c, sp = (ctypes.c_int * 3)(), (ctypes.c_int * 3)()
    _check(load().se_rs_cells_box(sides, float(rc), int(n_max), int(cells_per_rc), c, sp), "se_rs_cells_box")
    return tuple(c), tuple(sp)


def se_rs_plan_create_box(D, Ls, xi, rc, n_max, prec, cells_per_rc=0, stream=0):
    plan = ctypes.c_void_p()
    sides = (ctypes.c_double * 3)(*[float(v) for v in Ls])
    _check(load().se_rs_plan_create_box(int(D), sides, float(xi), float(rc), int(n_max), int(prec),
                                        int(cells_per_rc), ctypes.c_void_p(stream), ctypes.byref(plan)),
           "se_rs_plan_create_box")
    return plan


def se_rs_get_info(plan):
    c, sp, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
    _check(load().se_rs_get_info(plan, ctypes.byref(c), ctypes.byref(sp), ctypes.byref(b)), "se_rs_get_info")
    return c.value, sp.value, b.value


def se_rs_eval(plan, N, xyz_ptr, q_ptr, phi_ptr, force_ptr, energy_ptr, flags, stream) -> int:
    """Returns the status (callers decide whether to raise)."""
    return load().se_rs_eval(plan, int(N), ctypes.c_void_p(xyz_ptr), ctypes.c_void_p(q_ptr),
                             ctypes.c_void_p(phi_ptr), ctypes.c_void_p(force_ptr), ctypes.c_void_p(energy_ptr),
                             ctypes.c_uint(flags), ctypes.c_void_p(stream))


def se_rs_plan_profile(plan, stream, reset=True):
    """Records {name, launches, ms_total, ms_avg} of rs_cells, rs_pairs, rs_energy."""
    arr = (se_stage_record * 4)()
    n = ctypes.c_int()
    _check(load().se_rs_plan_profile(plan, ctypes.c_void_p(stream), arr, 4, ctypes.byref(n), int(reset)),
           "se_rs_plan_profile")
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, ms_total=arr[i].ms_total,
                 ms_avg=arr[i].ms_total / max(arr[i].launches, 1)) for i in range(n.value)]


def se_rs_plan_destroy(plan) -> int:
    return load().se_rs_plan_destroy(plan)


def se_batch_plan_destroy(plan) -> int:
    return load().se_batch_plan_destroy(plan)


def se_plan_destroy(plan) -> int:
    return load().se_plan_destroy(plan)


def declared_functions(header: str | None = None):
    """Names of the functions declared in include/se.h."""
    import re
    if header is None:
        header = os.path.join(os.path.dirname(_HERE), "include", "se.h")
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(se_\w+)\s*\(", text, re.M)))
