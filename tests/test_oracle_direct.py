"""Pins of the direct FP64 Ewald oracle (oracle/ewald_direct.cpp) against
facts that do not come from the oracle itself: lattice Madelung constants,
brute-force Coulomb sums, invariances of the Ewald split, finite differences,
library special functions and numerical quadrature of the paper's explicit
Fourier integrals (Eqs. fourier_space_explicit_2P / _1P)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as wl
from oracle import direct

OFF = np.array([0.1234, 0.2345, 0.3456])   # generic shift avoiding symmetric points


def _lattice(D, L=1.0):
    """Alternating +-1 lattice with spacing a = L/2: rock salt (3P), square
    checkerboard in one plane (2P), alternating chain (1P)."""
    a = L / 2
    pts, qs = [], []
    rng = {3: (2, 2, 2), 2: (2, 2, 1), 1: (2, 1, 1)}[D]
    for i in range(rng[0]):
        for j in range(rng[1]):
            for k in range(rng[2]):
                pts.append((np.array([i, j, k]) * a + OFF) % L)
                qs.append((-1.0) ** (i + j + k))
    return np.array(pts), np.array(qs), a


# Madelung constants: rock salt 1.747564594633 (3D), square lattice
# 1.615542626713 (2D), alternating chain 2 ln 2 (1D).
@pytest.mark.parametrize("D,const", [(3, 1.747564594633182), (2, 1.615542626712880),
                                     (1, 2.0 * math.log(2.0))])
@pytest.mark.parametrize("xi", [3.0, 6.0])
def test_madelung(D, const, xi):
    x, q, a = _lattice(D)
    phi, _ = direct.total(D, 1.0, xi, x, q)
    np.testing.assert_allclose(-phi * a / q, const, rtol=0, atol=2e-11)


def test_free_space_split_equals_coulomb():
    """0P: phi^R + phi^F + phi^self equals the plain Coulomb sum."""
    x, q = wl.system(60, 1.0, 7, "uniform")
    for xi in (3.0, 9.0):
        phi, g = direct.total(0, 1.0, xi, x, q)
        pc, gc = direct.coulomb_free(x, q)
        np.testing.assert_allclose(phi, pc, rtol=1e-12, atol=1e-11)
        np.testing.assert_allclose(g, gc, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_xi_invariance(D):
    """The total potential does not depend on xi (Section 2)."""
    x, q = wl.system(16, 1.0, 11 + D, "uniform")
    p1, g1 = direct.total(D, 1.0, 3.0, x, q)
    p2, g2 = direct.total(D, 1.0, 7.0, x, q)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-12 * np.abs(p1).max())
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-11 * np.abs(g1).max())


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_translation_invariance(D):
    x, q = wl.system(12, 1.0, 21 + D, "uniform")
    shift = np.array([0.31, -0.17, 0.05])
    xs = x + shift
    for d in range(D):                # wrap the periodic directions
        xs[:, d] %= 1.0
    p1, _ = direct.kspace(D, 1.0, 5.0, x, q)
    p2, _ = direct.kspace(D, 1.0, 5.0, xs, q)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-12 * np.abs(p1).max())


def _energy(fn, x, q):
    phi = fn(x)
    return 0.5 * float(np.dot(q, phi))


@pytest.mark.parametrize("D", [3, 2, 1, 0])
@pytest.mark.parametrize("part", ["kspace", "real"])
def test_force_is_minus_grad_energy(D, part):
    """q_m grad phi_m = dE/dx_m for E = 1/2 sum q phi, by central differences."""
    x, q = wl.system(10, 1.0, 31 + D, "uniform")
    xi = 5.0
    if part == "kspace":
        fn = lambda y: direct.kspace(D, 1.0, xi, y, q)[0]
        _, g = direct.kspace(D, 1.0, xi, x, q)
    else:
        rc = direct.real_space_cutoff(xi)
        fn = lambda y: direct.real_space(D, 1.0, xi, rc, y, q)[0]
        _, g = direct.real_space(D, 1.0, xi, rc, x, q)
    eps = 1e-5
    for m in (0, 3, 7):
        for d in range(3):
            xp = x.copy(); xp[m, d] += eps
            xm = x.copy(); xm[m, d] -= eps
            fd = (_energy(fn, xp, q) - _energy(fn, xm, q)) / (2 * eps)
            assert abs(fd - q[m] * g[m, d]) <= 1e-6 * max(1.0, abs(fd))


def test_incomplete_bessel_identities():
    """K0(a,b) + K0(b,a) = 2 K_0(2 sqrt(ab)) (the complete modified Bessel
    function), K0(a,0) = E1(a), and dK0/db by differences."""
    for a, b in [(0.02, 0.5), (0.3, 2.0), (1.5, 0.01), (0.005, 40.0), (3.0, 3.0)]:
        k_ab, d_ab = direct.incomplete_k0(a, b)
        k_ba, _ = direct.incomplete_k0(b, a)
        assert abs(k_ab + k_ba - 2.0 * special.k0(2.0 * math.sqrt(a * b))) <= 1e-13 * max(1, k_ab)
        h = 1e-6 * max(b, 1e-3)
        fd = (direct.incomplete_k0(a, b + h)[0] - direct.incomplete_k0(a, b - h)[0]) / (2 * h)
        assert abs(fd - d_ab) <= 1e-7 * max(1.0, abs(d_ab))
    for a in (0.01, 0.3, 2.0, 10.0):
        assert abs(direct.incomplete_k0(a, 0.0)[0] - special.exp1(a)) <= 1e-13 * special.exp1(a)


def test_ein_against_library():
    for xval in (1e-6, 0.1, 0.9, 1.0, 3.0, 30.0):
        ref = np.euler_gamma + math.log(xval) + special.exp1(xval)
        assert abs(direct.ein(xval) - ref) <= 1e-14 * max(1.0, abs(ref))


def _pair_system():
    # A neutral pair so that the k = 0 integrals converge.
    x = np.array([[0.21, 0.33, 0.40], [0.68, 0.59, 0.77]])
    q = np.array([1.0, -1.0])
    return x, q


def test_2p_closed_forms_against_quadrature():
    """Eq. (fourier_space_explicit_2P) integrated numerically over kappa_3
    for every periodic mode equals the closed forms (2pno0) [read with '+']
    and (2p0) used by the oracle."""
    x, q = _pair_system()
    L, xi = 1.0, 2.0
    nmax = direct.kspace_nmax(L, xi, 1e-16)
    phi, _ = direct.kspace(2, L, xi, x, q, nmax=nmax)
    m = 0
    tot = 0.0
    dk = 2 * math.pi / L
    for a in range(-nmax, nmax + 1):
        for b in range(-nmax, nmax + 1):
            k1, k2 = a * dk, b * dk
            k2sum = k1 * k1 + k2 * k2

            def f(kap):
                s = 0.0
                for n in range(2):
                    v = x[m] - x[n]
                    s += q[n] * math.cos(k1 * v[0] + k2 * v[1] + kap * v[2])
                return math.exp(-(k2sum + kap * kap) / (4 * xi * xi)) / (k2sum + kap * kap) * s \
                    if k2sum + kap * kap > 0 else 0.0

            if k2sum == 0:
                # neutral pair: the integrand is finite at kappa = 0; split off the origin
                val = 2 * integrate.quad(f, 1e-9, 60 * xi, limit=400, epsabs=1e-14)[0]
            else:
                val = 2 * integrate.quad(f, 0, 60 * xi, limit=400, epsabs=1e-14)[0]
            tot += 4 * math.pi / (2 * math.pi * L * L) * val
    assert abs(tot - phi[0]) <= 1e-8 * max(1.0, abs(phi[0]))


def test_1p_closed_forms_against_quadrature():
    """Eq. (fourier_space_explicit_1P), with the kappa-plane integral done
    radially (int d^2kappa e^{i kappa.w} g(|kappa|) = 2 pi int J0(kappa rho) g kappa dkappa),
    equals the closed forms (1pno0) and (1p0)."""
    x, q = _pair_system()
    L, xi = 1.0, 2.0
    nmax = direct.kspace_nmax(L, xi, 1e-16)
    phi, _ = direct.kspace(1, L, xi, x, q, nmax=nmax)
    m = 0
    dk = 2 * math.pi / L
    tot = 0.0
    for a in range(-nmax, nmax + 1):
        k1 = a * dk

        def f(kap):
            s = 0.0
            for n in range(2):
                v = x[m] - x[n]
                rho = math.hypot(v[1], v[2])
                s += q[n] * math.cos(k1 * v[0]) * special.j0(kap * rho)
            den = k1 * k1 + kap * kap
            return math.exp(-den / (4 * xi * xi)) / den * s * kap if den > 0 else 0.0

        val = 2 * math.pi * integrate.quad(f, 1e-12, 60 * xi, limit=800, epsabs=1e-14)[0]
        tot += 4 * math.pi / ((2 * math.pi) ** 2 * L) * val
    assert abs(tot - phi[0]) <= 1e-8 * max(1.0, abs(phi[0]))


# --- rectangular triply periodic boxes ---------------------------------------

@pytest.mark.parametrize("xi", [3.0, 6.0])
@pytest.mark.parametrize("reps", [(1, 1, 2), (2, 1, 3)])
def test_box_madelung_rock_salt(xi, reps):
    """Rock salt in a rectangular box made of reps[d] cubic cells of side 1
    per direction: the Madelung constant per ion is the cube's."""
    x1, q1, a = _lattice(3)
    pts, qs = [], []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                pts.append(x1 + np.array([i, j, k], dtype=float))
                qs.append(q1)
    x, q = np.concatenate(pts), np.concatenate(qs)
    phi, g = direct.total_box3(np.array(reps, dtype=float), xi, x, q)
    np.testing.assert_allclose(-phi * a / q, 1.747564594633182, rtol=0, atol=2e-11)
    np.testing.assert_allclose(g, 0.0, atol=1e-9)   # every ion sits at a symmetric site


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_box_supercell_matches_cube(axis):
    """A periodic system described by two copies of its cubic cell in a box
    twice as long along one axis is the same system: each part of the split
    (real space and Fourier space separately) at the original charges equals
    the cube's (only the even modes along that axis carry a structure
    factor)."""
    x, q = wl.system(24, 1.0, 70 + axis, "uniform")
    shift = np.zeros(3)
    shift[axis] = 1.0
    x2, q2 = np.concatenate([x, x + shift]), np.concatenate([q, q])
    Ls = np.ones(3)
    Ls[axis] = 2.0
    xi = 5.0
    tg = np.arange(len(q))
    pk, gk = direct.kspace(3, 1.0, xi, x, q)
    pk2, gk2 = direct.kspace_box3(Ls, xi, x2, q2, targets=tg)
    np.testing.assert_allclose(pk2, pk, rtol=0, atol=1e-12 * np.abs(pk).max())
    np.testing.assert_allclose(gk2, gk, rtol=0, atol=1e-11 * np.abs(gk).max())
    rc = direct.real_space_cutoff(xi)
    pr, gr = direct.real_space(3, 1.0, xi, rc, x, q)
    pr2, gr2 = direct.real_space_box3(Ls, xi, rc, x2, q2, targets=tg)
    np.testing.assert_allclose(pr2, pr, rtol=0, atol=1e-12 * np.abs(pr).max())
    np.testing.assert_allclose(gr2, gr, rtol=0, atol=1e-11 * np.abs(gr).max())


def test_box_xi_invariance():
    """In a rectangular box the total potential does not depend on xi."""
    x, q = wl.system(20, 1.0, 91, "uniform")
    x = x * np.array([1.0, 0.75, 1.5])
    Ls = np.array([1.0, 0.75, 1.5])
    p1, g1 = direct.total_box3(Ls, 4.0, x, q)
    p2, g2 = direct.total_box3(Ls, 8.0, x, q)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-12 * np.abs(p1).max())
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-11 * np.abs(g1).max())


@pytest.mark.parametrize("xi", [3.0, 6.0])
@pytest.mark.parametrize("reps", [(1, 2), (3, 1)])
def test_box2_madelung_square_lattice(xi, reps):
    """The alternating square lattice (spacing 1/2, one layer, z free) in a
    doubly periodic rectangular cell of reps[0] x reps[1] unit cells: the
    Madelung constant per ion is the square cell's."""
    a = 0.5
    off = np.array([0.1234, 0.2345, 0.3456])
    pts, qs = [], []
    for i in range(2 * reps[0]):
        for j in range(2 * reps[1]):
            pts.append(np.array([i * a + off[0], j * a + off[1], off[2]]))
            qs.append((-1.0) ** (i + j))
    x, q = np.array(pts), np.array(qs)
    phi, g = direct.total_box2(np.array(reps, dtype=float), xi, x, q)
    np.testing.assert_allclose(-phi * a / q, 1.615542626712880, rtol=0, atol=2e-11)
    np.testing.assert_allclose(g, 0.0, atol=1e-9)


@pytest.mark.parametrize("axis", [0, 1])
def test_box2_supercell_matches_square_cell(axis):
    """Two copies of a 2P unit cell in a cell twice as long along a periodic
    axis: each part of the split at the original charges equals the square
    cell's (the free direction untouched)."""
    x, q = wl.system(20, 1.0, 170 + axis, "uniform")
    shift = np.zeros(3)
    shift[axis] = 1.0
    x2, q2 = np.concatenate([x, x + shift]), np.concatenate([q, q])
    Ls = np.ones(2)
    Ls[axis] = 2.0
    xi = 5.0
    tg = np.arange(len(q))
    pk, gk = direct.kspace(2, 1.0, xi, x, q)
    pk2, gk2 = direct.kspace_box2(Ls, xi, x2, q2, targets=tg)
    np.testing.assert_allclose(pk2, pk, rtol=0, atol=1e-12 * np.abs(pk).max())
    np.testing.assert_allclose(gk2, gk, rtol=0, atol=1e-11 * np.abs(gk).max())
    rc = direct.real_space_cutoff(xi)
    pr, gr = direct.real_space(2, 1.0, xi, rc, x, q)
    pr2, gr2 = direct.real_space_box2(Ls, xi, rc, x2, q2, targets=tg)
    np.testing.assert_allclose(pr2, pr, rtol=0, atol=1e-12 * np.abs(pr).max())
    np.testing.assert_allclose(gr2, gr, rtol=0, atol=1e-11 * np.abs(gr).max())


def test_box2_xi_invariance():
    """For a rectangular 2P cell the total potential does not depend on xi."""
    x, q = wl.system(20, 1.0, 191, "uniform")
    x = x * np.array([1.0, 0.6, 1.0])
    Ls = np.array([1.0, 0.6])
    p1, g1 = direct.total_box2(Ls, 4.0, x, q)
    p2, g2 = direct.total_box2(Ls, 8.0, x, q)
    np.testing.assert_allclose(p1, p2, rtol=0, atol=1e-12 * np.abs(p1).max())
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-11 * np.abs(g1).max())
