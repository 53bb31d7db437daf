"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/se.h declares, applies the paper's parameter rules, and
rejects invalid arguments before touching the device."""
import ctypes
import math

import pytest

from oracle import se_discrete as se
from paper_1712_04732_amd import _lib as L

L_ = L


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = L.declared_functions()
    assert set(names) >= {"se_params_default", "se_plan_create", "se_plan_get_info", "se_eval",
                          "se_get_device_status", "se_plan_destroy", "se_status_string"}
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for s in range(10):
        assert L.se_status_string(s) != "unknown status"
    assert L.se_status_string(10) == "unknown status"
    assert "neutral" in L.se_status_string(L.SE_ERR_NONNEUTRAL)


@pytest.mark.parametrize("D,M,N,xi,kind", [(2, 96, 100000, 33.84, "pm1"), (1, 160, 1000000, 56.40, "normal"),
                                           (2, 32, 1000, 8.0, "uniform"), (1, 40, 300, 10.0, "uniform")])
def test_aft_estimates_match_oracle(D, M, N, xi, kind):
    """s and n_l of Eqs. (estimate-s), (estimate-nl) from the library equal the
    oracle's independent implementation (relative tolerance 1e-6 B)."""
    Q = float(N) if kind != "uniform" else N / 3.0
    B = se.B_scale(Q, xi, 1.0)
    eps = 1e-6 * B
    p = L.se_params_default(D, 1.0, xi, M, 8, L.SE_WIN_PKB, Q, eps, L.SE_F32)
    o = se.with_aft_estimates(D, 1.0, xi, M, 8, Q, eps, window="pkb")
    assert abs(p.s - o.s) < 1e-12 and p.n_l == o.n_l
    assert p.lambda_ == o.lam and p.s0 == o.s0 and p.shape == o.shape and p.nu == o.nu


def test_survey_aft_values():
    """Doubly periodic, M = 96, N = 1e5 +-1 charges, xi = 33.84, 1e-6 relative:
    s = 2.471 and n_l = 8; singly periodic M = 160, N = 1e6, xi = 56.40: s = 2.745,
    n_l = 16."""
    p = L.se_params_default(2, 1.0, 33.84, 96, 8, L.SE_WIN_PKB, 1e5, 1e-6 * se.B_scale(1e5, 33.84, 1.0), L.SE_F32)
    assert abs(p.s - 2.471) < 2e-3 and p.n_l == 8
    p = L.se_params_default(1, 1.0, 56.40, 160, 8, L.SE_WIN_PKB, 1e6, 1e-6 * se.B_scale(1e6, 56.40, 1.0), L.SE_F32)
    assert abs(p.s - 2.745) < 2e-3 and p.n_l == 16


@pytest.mark.parametrize("D,Lb,xi,M,P", [(4, 1.0, 5.0, 32, 8), (3, 0.0, 5.0, 32, 8), (3, 1.0, -1.0, 32, 8),
                                         (3, 1.0, 5.0, 33, 8), (3, 1.0, 5.0, 32, 7), (3, 1.0, 5.0, 8, 10),
                                         (3, 1.0, 5.0, 38, 8), (3, 1.0, 5.0, 32, 18), (3, float("nan"), 5.0, 32, 8)])
def test_plan_create_rejects_invalid_parameters(D, Lb, xi, M, P):
    """Section 3.3: M, P even, P <= M; M must factor into 2, 3, 5, 7 (38 = 2*19
    does not); the support is limited to P <= 16."""
    lib = L.load()
    p = L.se_params()
    p.D, p.L, p.xi, p.M, p.P, p.window = D, Lb, xi, M, P, L.SE_WIN_PKB
    plan = ctypes.c_void_p()
    assert lib.se_plan_create(ctypes.byref(p), 10, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert not plan.value


@pytest.mark.parametrize("D,My,Mz", [(2, 0, 30), (2, 30, 30), (1, 30, 0), (1, 0, 30), (0, 30, 30), (3, 31, 0),
                                     (3, 0, 38), (3, 6, 0), (2, 31, 0), (2, 6, 0)])
def test_plan_create_rejects_invalid_rectangular_boxes(D, My, Mz):
    """Rectangular cells are triply periodic boxes (My, Mz) or doubly periodic
    cells (My only), with even, 7-smooth grid lengths of at least P."""
    lib = L.load()
    p = L.se_params()
    p.D, p.L, p.xi, p.M, p.P, p.window = D, 1.0, 5.0, 32, 8, L.SE_WIN_PKB
    p.My, p.Mz = My, Mz
    plan = ctypes.c_void_p()
    assert lib.se_plan_create(ctypes.byref(p), 10, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert not plan.value


def test_null_arguments():
    lib = L.load()
    assert lib.se_plan_create(None, 10, None, None) == L.SE_ERR_ARG
    assert lib.se_eval(None, 0, None, None, None, None, None, 0, None) == L.SE_ERR_ARG
    assert lib.se_plan_get_info(None, None) == L.SE_ERR_ARG
    assert lib.se_plan_destroy(None) == L.SE_OK
    assert lib.se_params_default(3, 1.0, 5.0, 32, 8, 1, 1.0, 1e-6, 0, None) == L.SE_ERR_ARG
    out = L.se_params()
    assert lib.se_params_default(3, 1.0, 5.0, 32, 8, 1, 1.0, -1.0, 0, ctypes.byref(out)) == L.SE_ERR_PARAM


@pytest.mark.parametrize("D,L,N,tol", [(3, 1.0, 1000, 1e-7), (2, 0.7, 5000, 1e-7), (1, 1.9, 800, 1e-6),
                                       (0, 1.3, 20000, 1e-8), (3, 0.5, 40000, 1e-7)])
def test_params_for_tolerance_matches_oracle_rule(D, L, N, tol):
    """Section 6: M is the smallest even 7-smooth size whose Kolafa-Perram
    estimate over B meets the tolerance, with no error pollution
    (P <= f_W(M/(xi L))); recomputed here from the oracle's own estimates."""
    xi = 1.2 * N ** (1 / 3) / L
    Q = float(N)
    p = L_.se_params_for_tolerance(D, L, xi, Q, tol, 8, L_.SE_WIN_PKB, L_.SE_F32)
    B = se.B_scale(Q, xi, L)
    M = 8
    while True:
        M = se.smooth_even_up(M)
        if se.kp_kspace_error(Q, xi, L, M) <= tol * B and 8 <= se.pollution_bound("pkb", M / (xi * L)):
            break
        M += 2
    assert p.M == M
    if D in (1, 2):
        o = se.with_aft_estimates(D, L, xi, M, 8, Q, tol * B, window="pkb")
        assert abs(p.s - o.s) < 1e-12 and p.n_l == o.n_l


@pytest.mark.parametrize("tile3,fft_cap", [((6, 4, 4), 0), ((4, 4, 36), 0), ((8, 8, 8), 3000), ((8, 8, 8), 512),
                                           ((8, 8, 8), 16384)])
def test_plan_create_rejects_invalid_knobs(tile3, fft_cap):
    """Tile edges are multiples of 4 up to 32; FFT samples per workgroup a power
    of two in 1024..8192."""
    lib = L.load()
    p = L.se_params()
    p.D, p.L, p.xi, p.M, p.P, p.window = 3, 1.0, 5.0, 32, 8, L.SE_WIN_PKB
    for d in range(3):
        p.tile3[d] = tile3[d]
    p.fft_cap = fft_cap
    plan = ctypes.c_void_p()
    assert lib.se_plan_create(ctypes.byref(p), 10, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert not plan.value


def test_autotune_null_arguments():
    lib = L.load()
    p = L.se_params()
    assert lib.se_autotune(None, 10, None, None, 0, None, None, None) == L.SE_ERR_ARG
    assert lib.se_autotune(ctypes.byref(p), 0, None, None, 0, None, ctypes.byref(p), None) == L.SE_ERR_ARG
    assert lib.se_batch_autotune(None, None, 0, None, None, 0, None, None, None) == L.SE_ERR_ARG


@pytest.mark.parametrize("L,rc,n_max,k", [(1.0, 0.071, 10**6, 0), (1.0, 0.3, 1000, 2), (1.0, 2.5, 64, 1),
                                          (2.0, 0.5, 64, 1), (1.0, 1e-4, 10**7, 8), (1.0, 0.2, 3400, 3),
                                          (3.0, 1.0, 0, 0), (1.0, 1.0 / 3.0, 27, 1)])
def test_real_space_cells_cover_the_cutoff(L, rc, n_max, k):
    """Cell list of the real-space sum: s cells of side L/c reach rc and s - 1
    do not; c follows the cells-per-cutoff, charge-count and 160 limits."""
    c, s = L_.se_rs_cells(L, rc, n_max, k)
    h = L / c
    assert 1 <= c <= 160 and s >= 1
    assert s * h >= rc and (s == 1 or (s - 1) * h < rc)
    kk = 2 if k <= 0 else k
    assert c == max(1, min(math.floor(kk * L / rc), math.floor(max(1, n_max) ** (1 / 3) + 1e-9), 160))


@pytest.mark.parametrize("Ls,rc,n_max,k", [((1.0, 1.25, 0.75), 0.071, 10**6, 0), ((1.0, 2.0, 0.5), 0.3, 1000, 2),
                                           ((0.4, 1.0, 1.0), 0.5, 64, 1), ((1.0, 1.0, 3.0), 1e-4, 10**7, 8),
                                           ((2.0, 1.5, 1.0), 2.5, 0, 0), ((1.0, 0.5, 0.25), 0.01, 5000, 3)])
def test_real_space_box_cells_cover_the_cutoff(Ls, rc, n_max, k):
    """Rectangular box: per direction, s_d cells of side L_d/c_d reach rc and
    s_d - 1 do not; c_d follows the cells-per-cutoff, density and 160
    limits, with about one cell per charge at most."""
    c, s = L_.se_rs_cells_box(Ls, rc, n_max, k)
    kk = 2 if k <= 0 else k
    V = Ls[0] * Ls[1] * Ls[2]
    for d in range(3):
        h = Ls[d] / c[d]
        assert 1 <= c[d] <= 160 and s[d] >= 1
        assert s[d] * h >= rc and (s[d] == 1 or (s[d] - 1) * h < rc)
        by_n = max(1, math.floor(Ls[d] * (max(1, n_max) / V) ** (1 / 3) + 1e-9))
        assert c[d] == max(1, min(math.floor(kk * Ls[d] / rc), by_n, 160))
    assert c[0] * c[1] * c[2] <= max(1, n_max) * (1 + 1e-6) or min(c) == 1


@pytest.mark.parametrize("L", [1.0, 0.37, 3.0])
@pytest.mark.parametrize("rc,n_max,k", [(0.071, 10**6, 0), (0.3, 1000, 2), (2.5, 64, 1), (1e-4, 10**7, 8),
                                        (0.2, 3400, 3), (1.0 / 3.0, 27, 1), (0.05, 8000, 2)])
def test_real_space_box_cells_of_a_cube_match_the_cube(L, rc, n_max, k):
    """A rectangular box with equal sides gets the cube's cell list."""
    c, s = L_.se_rs_cells(L, rc * L, n_max, k)
    cb, sb = L_.se_rs_cells_box((L, L, L), rc * L, n_max, k)
    assert cb == (c, c, c) and sb == (s, s, s)


def test_real_space_cells_reject_invalid():
    lib = L.load()
    c, s = ctypes.c_int(), ctypes.c_int()
    for args in [(0.0, 0.1, 10, 0), (1.0, 0.0, 10, 0), (1.0, float("inf"), 10, 0), (1.0, 0.1, -1, 0),
                 (1.0, 0.1, 10, 9), (float("nan"), 0.1, 10, 0)]:
        assert lib.se_rs_cells(*args, ctypes.byref(c), ctypes.byref(s)) == L.SE_ERR_PARAM
    assert lib.se_rs_cells(1.0, 0.1, 10, 0, None, ctypes.byref(s)) == L.SE_ERR_ARG
    plan = ctypes.c_void_p()
    assert lib.se_rs_plan_create(4, 1.0, 1.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_plan_create(3, 1.0, -1.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_plan_create(3, 1.0, 1.0, 0.1, 10, 5, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    c3, s3 = (ctypes.c_int * 3)(), (ctypes.c_int * 3)()
    for Ls, rc, n, k in [((1.0, 0.0, 1.0), 0.1, 10, 0), ((1.0, 1.0, float("inf")), 0.1, 10, 0),
                         ((1.0, 1.0, 1.0), -0.1, 10, 0), ((1.0, 1.0, 1.0), 0.1, -1, 0),
                         ((1.0, 1.0, 1.0), 0.1, 10, 9), ((float("nan"), 1.0, 1.0), 0.1, 10, 0)]:
        sides = (ctypes.c_double * 3)(*Ls)
        assert lib.se_rs_cells_box(sides, rc, n, k, c3, s3) == L.SE_ERR_PARAM
        assert lib.se_rs_plan_create_box(3, sides, 1.0, rc, n, 0, k, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    sides = (ctypes.c_double * 3)(1.0, 2.0, 1.5)
    assert lib.se_rs_cells_box(None, 0.1, 10, 0, c3, s3) == L.SE_ERR_ARG
    assert lib.se_rs_cells_box(sides, 0.1, 10, 0, None, s3) == L.SE_ERR_ARG
    assert lib.se_rs_plan_create_box(3, None, 1.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_ARG
    assert lib.se_rs_plan_create_box(3, sides, 1.0, 0.1, 10, 0, 0, None, None) == L.SE_ERR_ARG
    assert lib.se_rs_plan_create_box(3, sides, 0.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_plan_create_box(3, sides, 1.0, 0.1, 10, 5, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_plan_create_box(4, sides, 1.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_plan_create_box(-1, sides, 1.0, 0.1, 10, 0, 0, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
    assert lib.se_rs_eval(None, 0, None, None, None, None, None, 0, None) == L.SE_ERR_ARG
    assert lib.se_rs_plan_destroy(None) == L.SE_OK


@pytest.mark.parametrize("Q,xi,Lb", [(1000.0, 13.18, 1.0), (1e6, 56.4, 1.0), (3.3e4, 3.0, 10.0), (40.0, 0.7, 2.0)])
def test_error_scale_matches_oracle(Q, xi, Lb):
    """B = sqrt(Q) f_c(xi L)/L of Section 5.2, against the oracle's own
    implementation of Eq. (fc-expression)."""
    assert abs(L.se_error_scale(Q, xi, Lb) / se.B_scale(Q, xi, Lb) - 1.0) < 1e-14


@pytest.mark.parametrize("Q,xi,Lb,tol", [(1000.0, 10.0, 1.0, 1e-6), (1e6, 56.4, 1.0, 1e-6), (4000.0, 6.0, 2.0, 1e-8),
                                         (3.3e4, 3.0, 10.0, 1e-12), (1e5, 33.84, 1.0, 1e-3)])
def test_real_space_cutoff_inverts_the_estimate(Q, xi, Lb, tol):
    """Eq. (KP_rc) is the exact inverse of Eq. (KP_real_space): the oracle's
    estimate at the library's cutoff equals the absolute tolerance tol B."""
    rc = L.se_rs_cutoff_for_tolerance(Lb, xi, Q, tol)
    est = se.kp_realspace_error(Q, xi, Lb, rc)
    assert abs(est / (tol * se.B_scale(Q, xi, Lb)) - 1.0) < 1e-9


def test_cutoff_and_scale_reject_invalid():
    lib = L.load()
    v = ctypes.c_double()
    assert lib.se_error_scale(1.0, 1.0, 1.0, None) == L.SE_ERR_ARG
    assert lib.se_error_scale(-1.0, 1.0, 1.0, ctypes.byref(v)) == L.SE_ERR_PARAM
    assert lib.se_error_scale(1.0, 0.0, 1.0, ctypes.byref(v)) == L.SE_ERR_PARAM
    assert lib.se_rs_cutoff_for_tolerance(1.0, 1.0, 1.0, 1e-6, None) == L.SE_ERR_ARG
    for args in [(0.0, 1.0, 1.0, 1e-6), (1.0, -1.0, 1.0, 1e-6), (1.0, 1.0, 0.0, 1e-6), (1.0, 1.0, 1.0, 0.0),
                 (1.0, float("nan"), 1.0, 1e-6)]:
        assert lib.se_rs_cutoff_for_tolerance(*args, ctypes.byref(v)) == L.SE_ERR_PARAM


@pytest.mark.parametrize("D,s0,ok", [(2, 1.99, False), (2, 2.0, True), (1, 2.40, False), (1, 2.42, True),
                                     (0, 2.70, False), (0, 1.9, False), (0, 2.74, True)])
def test_plan_create_enforces_the_upsampling_bound(D, s0, ok):
    """Section 3.4: s0 >= 1 + sqrt(d) for d = 3 - D free directions.  Below
    the bound the plan is rejected before any device work; at or above it
    validation passes (the call then needs a device, so only the rejection is
    checked here)."""
    lib = L.load()
    p = L.se_params()
    p.D, p.L, p.xi, p.M, p.P, p.window = D, 1.0, 5.0, 32, 8, L.SE_WIN_PKB
    p.s0, p.s, p.n_l = s0, 2.0, 2
    plan = ctypes.c_void_p()
    st = lib.se_plan_create(ctypes.byref(p), 10, None, ctypes.byref(plan))
    if ok:
        assert st != L.SE_ERR_PARAM
        if plan.value:
            lib.se_plan_destroy(plan)
    else:
        assert st == L.SE_ERR_PARAM and not plan.value


def test_workspace_and_adjoint_entries_reject_bad_arguments():
    """The workspace and adjoint calls validate their arguments on the host
    (no device work is enqueued for any of these)."""
    lib = L.load()
    b = ctypes.c_size_t()
    for fn in (lib.se_plan_workspace_size, lib.se_batch_plan_workspace_size, lib.se_rs_workspace_size):
        assert fn(None, ctypes.byref(b)) == L.SE_ERR_ARG
    for fn in (lib.se_plan_set_workspace, lib.se_batch_plan_set_workspace, lib.se_rs_set_workspace):
        assert fn(None, None, 0) == L.SE_ERR_ARG
    assert lib.se_eval_vjp(None, 0, None, None, None, None, None, None, 0, None) == L.SE_ERR_ARG
    # energy adjoint: bad precision, bad flags, missing inputs for a requested output
    assert lib.se_energy_vjp(4, 7, None, None, None, None, None, None, 0, None) == L.SE_ERR_ARG
    assert lib.se_energy_vjp(4, L.SE_F64, None, None, None, None, None, None, L.SE_ADD_SELF, None) == L.SE_ERR_ARG
    dummy = ctypes.c_void_p(4096)
    assert lib.se_energy_vjp(4, L.SE_F64, None, dummy, dummy, dummy, dummy, None, 0, None) == L.SE_ERR_ARG
    assert lib.se_energy_vjp(4, L.SE_F64, dummy, None, dummy, dummy, dummy, None, 0, None) == L.SE_ERR_ARG
    assert lib.se_energy_vjp(4, L.SE_F64, dummy, dummy, None, None, None, dummy, 0, None) == L.SE_ERR_ARG
    assert lib.se_energy_vjp(0, L.SE_F64, None, None, None, None, None, None, 0, None) == L.SE_OK


@pytest.mark.parametrize("D", [3, 2, 1, 0])
@pytest.mark.parametrize("window", ["pkb", "gaussian"])
def test_recipe_matches_oracle(D, window):
    """se_params_recipe (Section 6 with the error-pollution remedy) against
    the oracle's independent recipe over a grid of systems and tolerances."""
    w = L.SE_WIN_PKB if window == "pkb" else L.SE_WIN_GAUSSIAN
    lib = L.load()
    for Q, xi, Lb in ((3.32e4, 8.0, 1.0), (334.0, 6.0, 5.0), (31.4, 6.5, 1.0), (3.32e4, 3.0, 10.0)):
        for tol in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
            B = se.B_scale(Q, xi, Lb)
            ref = se.recipe(D, Lb, xi, Q, tol * B, window)
            out = L.se_params()
            st = lib.se_params_recipe(D, Lb, xi, Q, tol, w, L.SE_F64, ctypes.byref(out))
            if ref.P > 16:
                assert st == L.SE_ERR_PARAM
                continue
            assert st == L.SE_OK
            assert (out.M, out.P) == (ref.M, ref.P), (Q, xi, Lb, tol)
            assert out.nu == (ref.nu if window == "pkb" else 0)
            if D in (1, 2):
                assert out.n_l == ref.n_l and abs(out.s - ref.s) < 1e-12


def test_recipe_rejects_bad_arguments():
    lib = L.load()
    out = L.se_params()
    assert lib.se_params_recipe(3, 1.0, 8.0, 10.0, 1e-6, L.SE_WIN_PKB, L.SE_F64, None) == L.SE_ERR_ARG
    for args in ((4, 1.0, 8.0, 10.0, 1e-6), (3, -1.0, 8.0, 10.0, 1e-6), (3, 1.0, 0.0, 10.0, 1e-6),
                 (3, 1.0, 8.0, 0.0, 1e-6), (3, 1.0, 8.0, 10.0, 0.0), (3, 1.0, 8.0, 10.0, 1e-40)):
        assert lib.se_params_recipe(*args, L.SE_WIN_PKB, L.SE_F64, ctypes.byref(out)) == L.SE_ERR_PARAM


def test_es_window_rules():
    """The ES window takes beta = 2.5 P, no polynomial degree and the KB
    values of Table lambda; the W'_KB fit is refused for other windows."""
    lib = L.load()
    for D in (3, 2, 1, 0):
        p = L.se_params_default(D, 1.0, 8.0, 32, 8, L.SE_WIN_ES, 100.0, 1e-8, L.SE_F64)
        assert p.window == L.SE_WIN_ES and abs(p.shape - 20.0) < 1e-12 and p.nu == 0
        if D < 3:
            assert abs(p.lambda_ - (1.3 if D == 0 else 2.4)) < 1e-12
    p = L.se_params()
    p.D, p.L, p.xi, p.M, p.P, p.window, p.deriv_fit = 3, 1.0, 8.0, 32, 8, L.SE_WIN_ES, 1
    plan = ctypes.c_void_p()
    assert lib.se_plan_create(ctypes.byref(p), 10, None, ctypes.byref(plan)) == L.SE_ERR_PARAM
