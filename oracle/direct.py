"""Python face of the direct FP64 Ewald oracle (ewald_direct.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.

Functions return the Fourier-space potential phi^{D,F} of the paper's Eq.
(fourier_space_nonzero_ewald) and its gradient, the real-space part of Eq.
(real_space_ewald), the self term of Section 2, and the total potential of
Eq. (potential_split).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libse_oracle.so")
_SRC = os.path.join(_HERE, "ewald_direct.cpp")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP).  Returns the .so path."""
    if not force and os.path.exists(_SO):
        return _SO
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.oracle_real_space.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_long, dp, dp, ctypes.c_long,
                                          lp, dp, dp]
        lib.oracle_kspace.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_long, dp, dp, ctypes.c_long, lp, dp, dp]
        lib.oracle_coulomb_free.argtypes = [ctypes.c_long, dp, dp, ctypes.c_long, lp, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_real_space_box3.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp,
                                               ctypes.c_long, lp, dp, dp]
        lib.oracle_kspace_box3.argtypes = [dp, ctypes.c_double, ip, ctypes.c_long, dp, dp, ctypes.c_long, lp,
                                           dp, dp]
        lib.oracle_real_space_box2.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp,
                                               ctypes.c_long, lp, dp, dp]
        lib.oracle_kspace_box2.argtypes = [dp, ctypes.c_double, ip, ctypes.c_long, dp, dp, ctypes.c_long, lp,
                                           dp, dp]
        lib.oracle_incomplete_k0.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        lib.oracle_incomplete_k0.restype = None
        lib.oracle_ein.argtypes = [ctypes.c_double]
        lib.oracle_ein.restype = ctypes.c_double
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(x, q, targets):
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = q.shape[0]
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    return x, q, targets


def real_space(D, L, xi, rc, x, q, targets=None):
    """phi^R and grad phi^R at the targets (Eq. real_space_ewald), cutoff rc."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_real_space(D, L, xi, rc, q.shape[0], _dp(x), _dp(q), t.shape[0],
                                t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_real_space rejected its arguments")
    return phi, grad


def kspace_nmax(L, xi, tol=1e-18):
    """Largest |n| needed so that e^{-k^2/4xi^2} < tol beyond k = 2 pi n / L."""
    kmax = 2.0 * xi * math.sqrt(-math.log(tol))
    return int(math.ceil(kmax * L / (2.0 * math.pi)))


def kspace(D, L, xi, x, q, targets=None, nmax=None):
    """phi^{D,F} and its gradient at the targets, from the closed forms."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    if nmax is None:
        nmax = kspace_nmax(L, xi)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_kspace(D, L, xi, int(nmax), q.shape[0], _dp(x), _dp(q), t.shape[0],
                            t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_kspace rejected its arguments")
    return phi, grad


def coulomb_free(x, q, targets=None):
    """sum_{n != m} q_n / |x_m - x_n| and its gradient (Eq. potential, D = 0)."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    lib.oracle_coulomb_free(q.shape[0], _dp(x), _dp(q), t.shape[0],
                            t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(phi), _dp(grad))
    return phi, grad


def self_term(xi, q):
    """phi^self_m = -2 xi / sqrt(pi) q_m (Section 2)."""
    return -2.0 * xi / math.sqrt(math.pi) * np.asarray(q, dtype=np.float64)


def real_space_cutoff(xi, tol=1e-17):
    """A cutoff with erfc(xi rc) below tol: rc = sqrt(-log tol)/xi plus margin."""
    return math.sqrt(-math.log(tol)) / xi * 1.05


def total(D, L, xi, x, q, targets=None):
    """Total potential and gradient, Eq. (potential_split):
    phi = phi^R + phi^F + phi^self, all at the same xi."""
    x, q, t = _prep(x, q, targets)
    pr, gr = real_space(D, L, xi, real_space_cutoff(xi), x, q, t)
    pf, gf = kspace(D, L, xi, x, q, t)
    return pr + pf + self_term(xi, q[t]), gr + gf


def kspace_by_split(D, L, xi, x, q, targets=None, xi_o=None):
    """phi^{D,F}(xi) = phi_total(xi_o) - phi^R(xi) - phi^self(xi).

    The total potential does not depend on the splitting parameter (Section 2,
    after Eq. gamma), so a small xi_o keeps the k-space sums short while the
    real-space sum at the large xi is short-ranged.
    """
    x, q, t = _prep(x, q, targets)
    if xi_o is None:
        xi_o = max(2.0 / L, 1e-3)
    pt, gt = total(D, L, xi_o, x, q, t)
    pr, gr = real_space(D, L, xi, real_space_cutoff(xi), x, q, t)
    return pt - pr - self_term(xi, q[t]), gt - gr


def incomplete_k0(a, b):
    lib = _load()
    k0 = ctypes.c_double()
    d = ctypes.c_double()
    lib.oracle_incomplete_k0(a, b, ctypes.byref(k0), ctypes.byref(d))
    return k0.value, d.value


def ein(x):
    return _load().oracle_ein(x)


# --- triply periodic rectangular boxes (sides Ls = (L1, L2, L3)) -------------

def real_space_box3(Ls, xi, rc, x, q, targets=None):
    """phi^R and its gradient in the triply periodic box with sides Ls."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    Ls = np.ascontiguousarray(Ls, dtype=np.float64)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_real_space_box3(_dp(Ls), xi, rc, q.shape[0], _dp(x), _dp(q), t.shape[0],
                                     t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_real_space_box3 rejected its arguments")
    return phi, grad


def kspace_box3(Ls, xi, x, q, targets=None, tol=1e-18):
    """phi^{3P,F} and its gradient in the triply periodic box with sides Ls."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    Ls = np.ascontiguousarray(Ls, dtype=np.float64)
    nmax = np.ascontiguousarray([kspace_nmax(L, xi, tol) for L in Ls], dtype=np.int32)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_kspace_box3(_dp(Ls), xi, nmax.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), q.shape[0],
                                 _dp(x), _dp(q), t.shape[0], t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                 _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_kspace_box3 rejected its arguments")
    return phi, grad


def real_space_box2(Ls, xi, rc, x, q, targets=None):
    """phi^R and its gradient for the 2P lattice with rectangular cell Ls[0] x Ls[1]."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    Ls = np.ascontiguousarray(Ls[:2], dtype=np.float64)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_real_space_box2(_dp(Ls), xi, rc, q.shape[0], _dp(x), _dp(q), t.shape[0],
                                     t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_real_space_box2 rejected its arguments")
    return phi, grad


def kspace_box2(Ls, xi, x, q, targets=None, tol=1e-18):
    """phi^{2P,F} and its gradient for the rectangular 2P cell Ls[0] x Ls[1]."""
    lib = _load()
    x, q, t = _prep(x, q, targets)
    Ls = np.ascontiguousarray(Ls[:2], dtype=np.float64)
    nmax = np.ascontiguousarray([kspace_nmax(L, xi, tol) for L in Ls], dtype=np.int32)
    phi = np.zeros(t.shape[0])
    grad = np.zeros((t.shape[0], 3))
    rc_ = lib.oracle_kspace_box2(_dp(Ls), xi, nmax.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), q.shape[0],
                                 _dp(x), _dp(q), t.shape[0], t.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                 _dp(phi), _dp(grad))
    if rc_:
        raise ValueError("oracle_kspace_box2 rejected its arguments")
    return phi, grad


def total_box2(Ls, xi, x, q, targets=None):
    """phi (real + Fourier + self, Eq. potential_split) and its gradient for
    the 2P lattice with rectangular cell Ls[0] x Ls[1] (z free)."""
    rc = real_space_cutoff(xi)
    pr, gr = real_space_box2(Ls, xi, rc, x, q, targets)
    pk, gk = kspace_box2(Ls, xi, x, q, targets)
    q = np.asarray(q, dtype=np.float64)
    qs = q if targets is None else q[np.asarray(targets)]
    return pr + pk + self_term(xi, qs), gr + gk


def total_box3(Ls, xi, x, q, targets=None):
    """phi (real + Fourier + self, Eq. potential_split) and its gradient in
    the triply periodic box with sides Ls."""
    rc = real_space_cutoff(xi)
    pr, gr = real_space_box3(Ls, xi, rc, x, q, targets)
    pk, gk = kspace_box3(Ls, xi, x, q, targets)
    q = np.asarray(q, dtype=np.float64)
    qs = q if targets is None else q[np.asarray(targets)]
    return pr + pk + self_term(xi, qs), gr + gk
