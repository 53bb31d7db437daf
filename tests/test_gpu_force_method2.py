"""Force method 2 of Section 7.2 on the GPU (i k_d in the scaling step,
inverse transforms and a gathering with the window itself per direction),
against the discrete oracle's method 2 (same parameters: rounding only) and
the direct Ewald oracle's analytic gradient, and the paper's comparison with
method 1 (Fig. force: method 2 follows the potential's error curve, method 1
needs P + 2)."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct
from oracle import se_discrete as se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_04732_amd import SpectralEwald  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def run(plan, x, q, dtype=torch.float64, **kw):
    xt = torch.tensor(x, dtype=dtype, device=DEV)
    qt = torch.tensor(q, dtype=dtype, device=DEV)
    phi, g, E = plan(xt, qt, out_grad=True, **kw)
    torch.cuda.synchronize()
    return (phi.double().cpu().numpy() if phi is not None else None, g.double().cpu().numpy(),
            float(E) if E is not None else None)


def pair(D, M, P, xi=8.0, s=2.0, n_l=3, prec="f64", n_max=4096, nu=None):
    kw = dict(s=s, n_l=n_l) if D in (1, 2) else {}
    plan = SpectralEwald(D, 1.0, xi, M, P, prec=prec, n_max=n_max, force_method=2, nu=nu, **kw)
    p = se.Params(D=D, L=1.0, xi=xi, M=M, P=P, window="pkb", nu=nu, **kw)
    return plan, p


@pytest.mark.parametrize("D,M,P", [(3, 32, 8), (2, 24, 8), (1, 30, 6), (0, 24, 8), (3, 30, 10), (0, 28, 6)])
def test_method2_matches_discrete_oracle(D, M, P):
    print(f"case method2 vs O2 D={D} M={M} P={P}", flush=True)
    N = 1500
    x, q = wl.system(N, 1.0, 610 + D + M, "uniform")
    plan, p = pair(D, M, P, n_max=N)
    phi, g, E = run(plan, x, q)
    ref, gref = se.spectral_ewald(x, q, p, force_method=2)
    assert rel(phi, ref) < 1e-12
    assert rel(g, gref) < 1e-11
    assert abs(E - se.energy(q, ref)) < 1e-12 * abs(se.energy(q, ref))


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_method2_against_direct_forces(D):
    print(f"case method2 vs direct D={D}", flush=True)
    N = 300
    x, q = wl.system(N, 1.0, 700 + D, "uniform")
    Q = float((q * q).sum())
    B = se.B_scale(Q, 8.0, 1.0)
    pp = se.with_aft_estimates(D, 1.0, 8.0, 40, 16, Q, 1e-16 * B, window="pkb")
    kw = dict(s=pp.s, n_l=pp.n_l) if D in (1, 2) else {}
    plan = SpectralEwald(D, 1.0, 8.0, 40, 16, prec="f64", n_max=N, force_method=2, nu=9, **kw)
    _, g, _ = run(plan, x, q)
    _, gref = direct.kspace(D, 1.0, 8.0, x, q)
    assert rel(g, gref) < 1e-9


def test_potential_and_energy_unchanged_by_method():
    print("case method2 potential unchanged", flush=True)
    N = 2000
    x, q = wl.system(N, 1.0, 720, "pm1")
    a = SpectralEwald(3, 1.0, 8.0, 32, 8, prec="f64", n_max=N)
    b = SpectralEwald(3, 1.0, 8.0, 32, 8, prec="f64", n_max=N, force_method=2)
    pa, ga, Ea = run(a, x, q)
    pb, gb, Eb = run(b, x, q)
    assert np.array_equal(pa, pb) and Ea == Eb
    assert 0 < rel(gb, ga) < 1e-4
    # forces only: no potential pass is needed
    xt, qt = torch.tensor(x, device=DEV), torch.tensor(q, device=DEV)
    _, f, _ = b(xt, qt, phi=False, energy=False)
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), -q[:, None] * gb)


def test_fp32_method2_error():
    print("case method2 fp32", flush=True)
    N = 4000
    x, q = wl.system(N, 1.0, 730, "pm1")
    p64 = SpectralEwald(3, 1.0, 8.0, 64, 8, prec="f64", n_max=N, force_method=2)
    p32 = SpectralEwald(3, 1.0, 8.0, 64, 8, prec="f32", n_max=N, force_method=2)
    _, g64, _ = run(p64, x, q)
    _, g32, _ = run(p32, x, q, dtype=torch.float32)
    e = rel(g32, g64)
    print(f"method 2 FP32 vs FP64 grad: {e:.2e}")
    assert e < 5e-6


def test_fig_force_method1_needs_two_more_points():
    """Section 7.2, Fig. force (3P, L = 1, xi = 8, M = 64, PKB): through the
    HIP path, method 2's force error follows the potential's, method 1 is
    worse at equal P and recovers at P + 2."""
    print("case fig force", flush=True)
    N = 1000
    x, q = wl.system(N, 1.0, 740, "uniform")
    ref, gref = direct.kspace(3, 1.0, 8.0, x, q)
    for P in (6, 8, 10):
        m1 = SpectralEwald(3, 1.0, 8.0, 64, P, prec="f64", n_max=N)
        m2 = SpectralEwald(3, 1.0, 8.0, 64, P, prec="f64", n_max=N, force_method=2)
        m1p = SpectralEwald(3, 1.0, 8.0, 64, P + 2, prec="f64", n_max=N)
        phi, g1, _ = run(m1, x, q)
        _, g2, _ = run(m2, x, q)
        _, g1p, _ = run(m1p, x, q)
        e_phi, e1, e2, e1p = rel(phi, ref), rel(g1, gref), rel(g2, gref), rel(g1p, gref)
        print(f"P={P}: phi {e_phi:.2e} method 1 {e1:.2e} method 2 {e2:.2e} method 1 at P+2 {e1p:.2e}")
        assert e2 < 3 * e_phi and e_phi < 3 * e2
        assert e1 > 3 * e2
        assert e1p < 3 * e2
