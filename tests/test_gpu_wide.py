"""64-bit transform offsets.  A 3P FP64 plan at M = 840 has a z pass whose
workgroups span more than 4 GiB (n * z-stride * 16 B = 840 * 421 * 840 * 16 B),
so that pass addresses with 64-bit offsets; at M = 810 (810 * 406 * 810 * 16 B
< 2^32) every pass fits 32-bit offsets (both lengths are 7-smooth).  Both plans compute the same k-space potential to within the
method's error at P = 12 (xi L = 60 keeps the truncation error far below it),
so the wide path is checked against the narrow one on the same particles."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_04732_amd import SpectralEwald  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_wide_offsets_match_narrow_plan():
    print("case wide offsets M=840 vs M=810", flush=True)
    x, q = wl.system(200, 1.0, 4242, "pm1")
    xt, qt = torch.tensor(x, device=DEV), torch.tensor(q, device=DEV)
    out = {}
    for M, wide in ((810, 0), (840, 1 << 2)):
        plan = SpectralEwald(3, 1.0, 60.0, M, 12, prec="f64", n_max=200)
        assert plan.info.fft_wide == wide, (M, plan.info.fft_wide)
        phi, f, e = plan(xt, qt)
        torch.cuda.synchronize()
        out[M] = (phi.cpu().numpy(), f.cpu().numpy(), float(e))
        del plan
        torch.cuda.empty_cache()
    assert rel(out[840][0], out[810][0]) < 1e-7
    assert rel(out[840][1], out[810][1]) < 1e-6
    assert abs(out[840][2] - out[810][2]) <= 1e-7 * abs(out[810][2])
