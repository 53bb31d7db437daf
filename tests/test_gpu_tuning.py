"""Schedule knobs and the autotuner: every tile shape, FFT workgroup size and
XCD mapping the tuner can choose gives the discrete oracle's result, and a
tuned plan (single or batch) computes what the default plan computes."""
import numpy as np
import pytest

import workloads as wl
from oracle import se_discrete as se

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_04732_amd import SpectralEwald, SpectralEwaldBatch, _lib  # noqa: E402

DEV = torch.device("cuda:0")
TILES = [(16, 16, 16), (32, 16, 8), (32, 8, 8), (16, 16, 8), (16, 8, 8), (8, 8, 8), (8, 8, 4), (4, 4, 4)]


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _plan(D, M, N, knobs, prec="f64"):
    kw = {"s": 2.0, "n_l": 3} if D in (1, 2) else {}
    base = SpectralEwald(D, 1.0, 8.0, M, 8, prec=prec, n_max=N, **kw)
    p = base.params
    for k, v in knobs.items():
        if k == "tile3":
            for d in range(3):
                p.tile3[d] = v[d]
        else:
            setattr(p, k, v)
    return SpectralEwald.from_params(p, N), se.Params(D=D, L=1.0, xi=8.0, M=M, P=8, window="pkb", **kw)


def _eval(plan, x, q):
    phi, g, _ = plan(torch.tensor(x, device=DEV), torch.tensor(q, device=DEV), out_grad=True)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), g.double().cpu().numpy()


_ORACLE = {}


def _oracle(key, x, q, p):
    if key not in _ORACLE:
        _ORACLE[key] = se.spectral_ewald(x, q, p)
    return _ORACLE[key]


@pytest.mark.parametrize("D", [3, 2, 1, 0])
@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_every_tile_shape_matches_oracle(D, tile, mode):
    """M = 36 is a multiple of no tile edge above 4, so every shape has short
    last tiles in the periodic directions; all spreading modes (the column
    mode takes tiles with x*y <= 256 and z <= 16 only)."""
    print(f"case tile D={D} tile={tile} spread mode {mode}", flush=True)
    x, q = wl.system(600, 1.0, 40 + D, "uniform")
    if mode == 3 and (tile[0] * tile[1] > 256 or tile[2] > 16):
        with pytest.raises(_lib.SEError) as e:
            _plan(D, 36, 600, {"tile3": tile, "tile": 0, "spread_mode": mode})
        assert e.value.status == _lib.SE_ERR_PARAM
        return
    plan, p = _plan(D, 36, 600, {"tile3": tile, "tile": 0, "spread_mode": mode})
    assert tuple(plan.info.tile) == tile and plan.info.spread_mode == mode
    phi, g = _eval(plan, x, q)
    ref, gref = _oracle(("tile", D), x, q, p)
    assert rel(phi, ref) < 1e-12 and rel(g, gref) < 1e-11


@pytest.mark.parametrize("D", [3, 2, 1, 0])
@pytest.mark.parametrize("knobs", [dict(fft_cap=1024), dict(fft_cap=4096), dict(fft_cap=8192),
                                   dict(xcd_tiles=-1, xcd_fft=-1), dict(xcd_tiles=1, xcd_fft=-1)])
def test_fft_and_mapping_knobs_match_oracle(D, knobs):
    print(f"case knobs D={D} {knobs}", flush=True)
    x, q = wl.system(500, 1.0, 60 + D, "uniform")
    plan, p = _plan(D, 30, 500, knobs)
    phi, g = _eval(plan, x, q)
    ref, gref = _oracle(("knobs", D), x, q, p)
    assert rel(phi, ref) < 1e-12 and rel(g, gref) < 1e-11


@pytest.mark.parametrize("D,M", [(3, 42), (3, 70), (2, 30), (1, 36), (0, 28)])
@pytest.mark.parametrize("cap", [0, 1024, 4096])
def test_transform_blocks_of_any_pencil_count(D, M, cap):
    """Transform workgroups hold any number of pencils, chosen so that a
    pencil range splits into equal blocks, with partial blocks, odd counts
    and the real passes' pencil pairs (in place at the default cap and 1024,
    two alternating buffers at 4096): the discrete oracle's result in FP64
    and within the FP32 bounds."""
    print(f"case fft blocks D={D} M={M} cap={cap}", flush=True)
    x, q = wl.system(400, 1.0, 80 + D + M, "uniform")
    knobs = {"fft_cap": cap} if cap else {}
    plan, p = _plan(D, M, 400, knobs)
    blocks = list(plan.info.fft_block)
    print(f"  blocks per pass {blocks}")
    assert all(b >= 1 for b in blocks)
    if D == 3 and M == 70 and cap == 0:
        assert any(b & (b - 1) for b in blocks)   # not all powers of two
    phi, g = _eval(plan, x, q)
    ref, gref = _oracle(("blocks", D, M), x, q, p)
    assert rel(phi, ref) < 1e-12 and rel(g, gref) < 1e-11
    plan32, _ = _plan(D, M, 400, knobs, prec="f32")
    phi32, g32 = _eval(plan32, x, q)
    assert rel(phi32, ref) < 1e-5 and rel(g32, gref) < 2e-5


def test_invalid_knobs_rejected():
    base = SpectralEwald(3, 1.0, 8.0, 32, 8, prec="f64", n_max=10)
    for edit in (lambda p: setattr(p, "fft_cap", 3000), lambda p: setattr(p, "fft_cap", 512)):
        p = _lib.se_params()
        ctypes_copy(base.params, p)
        edit(p)
        with pytest.raises(_lib.SEError) as e:
            _lib.se_plan_create(p, 10, torch.cuda.current_stream().cuda_stream)
        assert e.value.status == _lib.SE_ERR_PARAM


def ctypes_copy(src, dst):
    import ctypes
    ctypes.memmove(ctypes.byref(dst), ctypes.byref(src), ctypes.sizeof(src))


@pytest.mark.parametrize("D", [3, 0])
def test_autotuned_plan_computes_the_same(D):
    print(f"case autotune D={D}", flush=True)
    N = 4000
    x, q = wl.system(N, 1.0, 80 + D, "pm1")
    base = SpectralEwald(D, 1.0, 10.0, 40, 8, prec="f64", n_max=N)
    xt, qt = torch.tensor(x, device=DEV), torch.tensor(q, device=DEV)
    tuned, rep = base.autotune(xt, qt)
    print(f"tuned tile {list(tuned.info.tile)} fft_cap {tuned.info.fft_cap} report {rep}")
    assert rep["candidates"] >= 2 and rep["ms_tuned"] <= rep["ms_default"] * 1.0001
    phi0, g0 = _eval(base, x, q)
    phi1, g1 = _eval(tuned, x, q)
    # the tile shape sets the per-tile fixed-point scale of the spreading, so
    # the two plans round differently: the FP64 bar of the oracle comparison
    assert rel(phi1, phi0) < 1e-12 and rel(g1, g0) < 1e-11


def test_batch_autotune_computes_the_same():
    print("case batch autotune", flush=True)
    rng = np.random.default_rng(11)
    params, N, xs, qs = [], [], [], []
    for i in range(8):
        D = [3, 2, 1, 0][i % 4]
        n = int(rng.integers(100, 900)) * 2
        Lb = float(rng.uniform(0.7, 1.4))
        x, q = wl.system(n, Lb, 300 + i, "pm1")
        params.append(_lib.se_params_for_tolerance(D, Lb, wl.batch_xi(n, Lb), float(n), 1e-7, 8,
                                                   _lib.SE_WIN_PKB, _lib.SE_F32))
        N.append(n)
        xs.append(x)
        qs.append(q)
    x = torch.tensor(np.concatenate(xs), device=DEV, dtype=torch.float32)
    q = torch.tensor(np.concatenate(qs), device=DEV, dtype=torch.float32)
    b0 = SpectralEwaldBatch(params, N)
    b1, rep = SpectralEwaldBatch.tuned(params, N, x, q)
    print(f"batch tuner report {rep}")
    assert rep["ms_tuned"] <= rep["ms_default"] * 1.0001
    r0 = [t.double().cpu().numpy() for t in b0(x, q, out_grad=True)]
    r1 = [t.double().cpu().numpy() for t in b1(x, q, out_grad=True)]
    # FP32: the tile shape changes the per-tile fixed-point scale and the FFT
    # workgroup size nothing; differences are FP32 rounding
    assert rel(r1[0], r0[0]) < 2e-6 and rel(r1[1], r0[1]) < 5e-6


@pytest.mark.parametrize("mode", [2, 3])
@pytest.mark.parametrize("D,M,P,tile", [(3, 10, 8, (16, 16, 16)), (2, 12, 10, (32, 8, 8)), (1, 14, 12, (8, 8, 8)),
                                        (3, 16, 16, (4, 4, 4)), (0, 12, 6, (16, 16, 8))])
def test_clipped_spread_small_periodic_grids(D, M, P, tile, mode):
    """Clipped spreading where a stencil wraps onto the same tile more than
    once (tiles wider than the periodic grid, supports close to M)."""
    print(f"case clip mode {mode} D={D} M={M} P={P} tile={tile}", flush=True)
    x, q = wl.system(300, 1.0, 90 + D, "uniform")
    kw = {"s": 2.0, "n_l": 2} if D in (1, 2) else {}
    base = SpectralEwald(D, 1.0, 4.0, M, P, prec="f64", n_max=300, **kw)
    p = base.params
    for d in range(3):
        p.tile3[d] = tile[d]
    p.tile, p.spread_mode = 0, mode
    plan = SpectralEwald.from_params(p, 300)
    assert plan.info.spread_mode == mode
    phi, g = _eval(plan, x, q)
    ref, gref = se.spectral_ewald(x, q, se.Params(D=D, L=1.0, xi=4.0, M=M, P=P, window="pkb", **kw))
    # the fixed-point quantum is 2^-50 times the sum of |q| over every stencil
    # visit of the tile; here each particle visits the one tile once per
    # periodic image it wraps onto (up to 2^3 times), so the bar is 10x the
    # single-visit FP64 bar
    assert rel(phi, ref) < 1e-11 and rel(g, gref) < 1e-10
