"""The paper's accuracy experiments through the HIP path (Section 5.2,
Section 6, Section 7.1), on seeded synthetic systems like the paper's
(positions uniform in the box, charges uniform in [-1, 1] re-centred), with
the direct Ewald oracle as reference:

  * Fig. AB_test: approximation error over B against 10 e^{-2.5P} (PKB) and
    2 e^{-(pi/2) P c} (Gaussian) over systems of several N, L, xi L and all
    four periodicities;
  * Fig. shape_parameter: the KB shape beta = 2.5 P near the minimum error;
  * Fig. error_pollution and the remedy of Section 5.2 (M + 5 %, P + 4), and
    the whole Section 6 recipe reaching its tolerance;
  * Fig. poldeg-vs-P: the degree rule nu = min(P/2 + 2, 9) as accurate as the
    exact KB window;
  * Fig. efficiency (left): about n digits at P = n with PKB and at
    P = 1.6 n with the Gaussian.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import direct
from oracle import se_discrete as se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_04732_amd import SpectralEwald, params_recipe  # noqa: E402

DEV = torch.device("cuda:0")


def gpu_phi(D, L, xi, M, P, window, x, q, **kw):
    """FP64 potential phi~^{D,F} of the HIP path (no self term)."""
    plan = SpectralEwald(D, L, xi, M, P, window=window, prec="f64", n_max=x.shape[0], **kw)
    phi, _, _ = plan(torch.tensor(x, device=DEV), torch.tensor(q, device=DEV), force=False, energy=False)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


def aft(D, L, xi, M, P, Q, eps, window):
    """s and n_l of the AFT from the estimates of Section 6 at tolerance eps."""
    if D not in (1, 2):
        return {}
    p = se.with_aft_estimates(D, L, xi, M, P, Q, eps, window=window)
    return {"s": p.s, "n_l": p.n_l}


def est(window, P):
    return 10 * math.exp(-2.5 * P) if window == "pkb" else 2 * math.exp(-(math.pi / 2) * P * math.sqrt(0.91))


def test_fig_ab_error_estimates():
    """Absolute rms error over B within a factor 4 of the estimates for every
    system, and within a factor 2.5 in the median (Fig. AB_test), with grids
    fine enough that truncation and pollution do not enter."""
    ratios = {}
    for D in (3, 2, 1, 0):
        for Lb in (1.0, 5.0):
            for xiL in (5.0, 15.0, 25.0):
                print(f"case AB D={D} L={Lb} xiL={xiL}", flush=True)
                xi = xiL / Lb
                x, q = wl.system(150, Lb, int(1000 + 10 * D + Lb + xiL), "uniform")
                Q = float((q * q).sum())
                B = se.B_scale(Q, xi, Lb)
                ref, _ = direct.kspace(D, Lb, xi, x, q)
                M = se.smooth_even_up(max(math.ceil(2 * se.kinf_for_tolerance(Q, xi, Lb, 1e-16 * B)),
                                          math.ceil(3.8 * xiL)))
                for win in ("pkb", "gaussian"):
                    for P in (4, 8, 12):
                        phi = gpu_phi(D, Lb, xi, M, P, win, x, q, **aft(D, Lb, xi, M, P, Q, 1e-16 * B, win))
                        r = math.sqrt(np.mean((phi - ref) ** 2)) / B / est(win, P)
                        ratios.setdefault((win, P), []).append(r)
                        assert 0.25 < r < 4.0, (D, Lb, xiL, win, P, r)
    for k, v in ratios.items():
        print(k, "median ratio %.2f" % np.median(v))
        assert 0.4 < np.median(v) < 2.5


def test_fig_shape_parameter():
    """KB (PKB with nu = 9) error against beta for P = 6, 10 (N = 100, L = 1,
    M = 28, xi = 6.5, 3P): the minimum lies between 2.25 P and 3 P, beta =
    2.5 P is within a factor 6 of it and below the estimate of Eq.
    (approx_error_KB) with C_KB = 100, and the error grows tenfold toward
    beta = 1.5 P and 3.5 P."""
    print("case shape parameter", flush=True)
    x, q = wl.system(100, 1.0, 91, "uniform")
    ref, _ = direct.kspace(3, 1.0, 6.5, x, q)
    from scipy import special
    for P in (6, 10):
        fs = (1.5, 1.75, 2.0, 2.25, 2.5, 2.75, 3.0, 3.25, 3.5)
        err = np.array([math.sqrt(np.mean((gpu_phi(3, 1.0, 6.5, 28, P, "pkb", x, q, shape=f * P, nu=9) - ref) ** 2))
                        for f in fs])
        print(P, " ".join("%.1e" % e for e in err))
        i = int(np.argmin(err))
        assert 2.25 <= fs[i] <= 3.0
        e25 = err[fs.index(2.5)]
        beta = 2.5 * P
        assert e25 < 6 * err[i]
        assert e25 < 100 * (math.exp(-2 * math.pi * P * P / beta) + special.erfc(math.sqrt(beta)))
        assert err[0] > 10 * e25 and err[-1] > 10 * e25


def test_fig_error_pollution_and_remedy():
    """3P, N = 1000, L = 5, xi = 6 (Fig. error_pollution): with P <= f_W(M/(xi
    L)) the error follows the estimate; above it the error stays well above
    the estimate (and above the truncation level); M + 5 % and P + 4 bring it
    down to the expected level."""
    x, q = wl.system(1000, 5.0, 92, "uniform")
    Q = float((q * q).sum())
    B = se.B_scale(Q, 6.0, 5.0)
    tg = np.arange(0, 1000, 4)
    ref, _ = direct.kspace(3, 5.0, 6.0, x, q, targets=tg)
    nref = np.linalg.norm(ref)

    def err(M, P, win="pkb"):
        return np.linalg.norm(gpu_phi(3, 5.0, 6.0, M, P, win, x, q)[tg] - ref) / nref

    for M in (70, 100):
        trunc = se.kp_kspace_error(Q, 6.0, 5.0, M) / B
        fw = se.pollution_bound("pkb", M / 30.0)
        for P in (4, 6, 8, 10, 12):
            e = err(M, P)
            print(f"case pollution M={M} P={P}: {e:.2e} (estimate {est('pkb', P):.1e}, f_W {fw:.2f})", flush=True)
            if P <= fw:
                assert e < 3 * max(est("pkb", P), trunc)
            elif est("pkb", P) > 10 * trunc or P >= fw + 1.5:
                assert e > 5 * max(est("pkb", P), trunc)
    for M, P in ((70, 8), (70, 10), (100, 12)):
        M2 = se.smooth_even_up(math.ceil(1.05 * M))
        e = err(M2, P + 4)
        print(f"case remedy M={M}->{M2} P={P}->{P + 4}: {e:.2e}", flush=True)
        assert e < 3 * max(est("pkb", P), se.kp_kspace_error(Q, 6.0, 5.0, M) / B)


@pytest.mark.parametrize("D", [3, 2, 0])
def test_section6_recipe_reaches_the_tolerance(D):
    """params_recipe (M, P from the tolerance, with the pollution remedy):
    the HIP path's error against the direct sum is within 3x the tolerance."""
    x, q = wl.system(400, 1.0, 94 + D, "uniform")
    Q = float((q * q).sum())
    ref, _ = direct.kspace(D, 1.0, 8.0, x, q)
    B = se.B_scale(Q, 8.0, 1.0)
    for tol in (1e-4, 1e-7, 1e-10):
        p = params_recipe(D, 1.0, 8.0, Q, tol)
        kw = {"s": p.s, "n_l": p.n_l} if D in (1, 2) else {}
        phi = gpu_phi(D, 1.0, 8.0, p.M, p.P, "pkb", x, q, **kw)
        e = math.sqrt(np.mean((phi - ref) ** 2)) / B
        print(f"case recipe D={D} tol={tol:g}: M={p.M} P={p.P} error/B {e:.2e}", flush=True)
        assert e < 3 * tol


def test_fig_poldeg_rule():
    """3P, L = 1, xi = 8, M = 32, beta = 2.5 P (Fig. poldeg-vs-P): the PKB
    window with nu = min(P/2 + 2, 9) is within 1.5x of the exact KB window's
    error (the oracle's KB) for every P, nu = 9 for all P, and a low degree
    stalls."""
    x, q = wl.system(2000, 1.0, 93, "uniform")
    tg = np.arange(0, 2000, 5)
    ref, _ = direct.kspace(3, 1.0, 8.0, x, q, targets=tg)
    nref = np.linalg.norm(ref)
    for P in (4, 6, 8, 10, 12, 14, 16):
        kb, _ = se.spectral_ewald(x, q, se.Params(D=3, L=1.0, xi=8.0, M=32, P=P, window="kb"), targets=tg,
                                  grad=False)
        e_kb = np.linalg.norm(kb - ref) / nref
        e_rule = np.linalg.norm(gpu_phi(3, 1.0, 8.0, 32, P, "pkb", x, q)[tg] - ref) / nref
        e9 = np.linalg.norm(gpu_phi(3, 1.0, 8.0, 32, P, "pkb", x, q, nu=9)[tg] - ref) / nref
        print(f"case poldeg P={P}: KB {e_kb:.2e} rule {e_rule:.2e} nu=9 {e9:.2e}", flush=True)
        assert e_rule < 1.5 * e_kb and e9 < 1.5 * e_kb
    e_low = np.linalg.norm(gpu_phi(3, 1.0, 8.0, 32, 12, "pkb", x, q, nu=4)[tg] - ref) / nref
    assert e_low > 1e3 * e9


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_fig_efficiency_digits(D):
    """L = 1, xi = 8, M = 32, other errors negligible (Fig. efficiency, left):
    about n digits at P = n with PKB and at P = 1.6 n with the Gaussian."""
    x, q = wl.system(600, 1.0, 95 + D, "uniform")
    Q = float((q * q).sum())
    B = se.B_scale(Q, 8.0, 1.0)
    ref, _ = direct.kspace(D, 1.0, 8.0, x, q)
    nref = np.linalg.norm(ref)
    for win, Ps in (("pkb", (4, 6, 8, 10, 12)), ("gaussian", (6, 10, 14, 16))):
        for P in Ps:
            phi = gpu_phi(D, 1.0, 8.0, 32, P, win, x, q, **aft(D, 1.0, 8.0, 32, P, Q, 1.5e-17 * B, win))
            digits = -math.log10(np.linalg.norm(phi - ref) / nref)
            n = P if win == "pkb" else P / 1.6
            print(f"case efficiency D={D} {win} P={P}: {digits:.1f} digits", flush=True)
            assert n - 2.0 < digits < n + 1.5
