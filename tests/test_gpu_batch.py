"""Batched evaluation (one launch per stage over all systems): every system of
a mixed batch (all four periodicities, uneven N) against the discrete oracle
and the single-system path."""
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


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _batch(n_sys, prec, seed=7):
    rng = np.random.default_rng(seed)
    systems, params = [], []
    for i in range(n_sys):
        D = [3, 2, 1, 0][i % 4]
        N = int(rng.integers(20, 700)) * 2
        L = float(rng.uniform(0.6, 1.6))
        x, q = wl.system(N, L, 1000 + i, "pm1")
        xi = wl.batch_xi(N, L)
        p = _lib.se_params_for_tolerance(D, L, xi, float(N), 1e-7, 8, _lib.SE_WIN_PKB,
                                         _lib.SE_F64 if prec == "f64" else _lib.SE_F32)
        systems.append(dict(D=D, N=N, L=L, xi=xi, x=x, q=q, M=p.M, s=p.s, n_l=p.n_l))
        params.append(p)
    return systems, params


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_matches_oracle_per_system(prec):
    print(f"case batch {prec}", flush=True)
    systems, params = _batch(12, prec)
    b = SpectralEwaldBatch(params, [s["N"] for s in systems])
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), device=DEV)
    q = torch.tensor(np.concatenate([s["q"] for s in systems]), device=DEV)
    phi, grad, E = b(x, q, out_grad=True)
    torch.cuda.synchronize()
    phi, grad, E = phi.double().cpu().numpy(), grad.double().cpu().numpy(), E.cpu().numpy()
    tol_phi, tol_g = (1e-12, 1e-11) if prec == "f64" else (2e-6, 5e-6)
    o = 0
    for k, s in enumerate(systems):
        kw = {"s": s["s"], "n_l": s["n_l"]} if s["D"] in (1, 2) else {}
        p = se.Params(D=s["D"], L=s["L"], xi=s["xi"], M=s["M"], P=8, window="pkb", **kw)
        ref, gref = se.spectral_ewald(s["x"], s["q"], p)
        sl = slice(o, o + s["N"])
        assert rel(phi[sl], ref) < tol_phi, (k, s["D"])
        assert rel(grad[sl], gref) < tol_g, (k, s["D"])
        Eref = se.energy(s["q"], ref)
        assert abs(E[k] - Eref) <= 10 * tol_phi * abs(Eref)
        o += s["N"]


def test_batch_equals_single_system_path():
    print("case batch vs single", flush=True)
    systems, params = _batch(8, "f64", seed=11)
    b = SpectralEwaldBatch(params, [s["N"] for s in systems])
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), device=DEV)
    q = torch.tensor(np.concatenate([s["q"] for s in systems]), device=DEV)
    phi, f, E = b(x, q)
    o = 0
    for k, s in enumerate(systems):
        kw = {"s": s["s"], "n_l": s["n_l"]} if s["D"] in (1, 2) else {}
        plan = SpectralEwald(s["D"], s["L"], s["xi"], s["M"], 8, prec="f64", n_max=s["N"], **kw)
        p1, f1, e1 = plan(torch.tensor(s["x"], device=DEV), torch.tensor(s["q"], device=DEV))
        sl = slice(o, o + s["N"])
        assert rel(phi[sl].cpu().numpy(), p1.cpu().numpy()) < 1e-13
        assert rel(f[sl].cpu().numpy(), f1.cpu().numpy()) < 1e-12
        assert abs(float(E[k]) - float(e1)) <= 1e-13 * abs(float(e1))
        o += s["N"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_evaluation_replays_from_a_graph(prec):
    """A batch evaluation captured in a graph (no memory set or copy nodes in
    the evaluation path) replays bit for bit what the eager call computes,
    on new inputs written in place between replays, with eager evaluations
    of the plan in between."""
    print(f"case batch graph {prec}", flush=True)
    systems, params = _batch(8, prec, seed=11)
    b = SpectralEwaldBatch(params, [s["N"] for s in systems])
    dt = torch.float32 if prec == "f32" else torch.float64
    x0 = np.concatenate([s["x"] for s in systems])
    q0 = np.concatenate([s["q"] for s in systems])
    x = torch.tensor(x0, dtype=dt, device=DEV)
    q = torch.tensor(q0, dtype=dt, device=DEV)
    out = b(x, q)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            b(x, q, out=out, check=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b(x, q, out=out, check=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for k in range(3):
        # new positions (a shift keeps each system in its box), same charges
        shift = rng.uniform(-0.01, 0.01, size=3)
        xs = x0.copy()
        off = 0
        for s_ in systems:
            xs[off:off + s_["N"]] = np.mod(s_["x"] + shift, s_["L"]) if s_["D"] == 3 else s_["x"]
            off += s_["N"]
        x.copy_(torch.tensor(xs, dtype=dt))
        ref = [t.clone() for t in b(x, q)]          # eager
        for t in out:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        for a, r in zip(out, ref):
            assert torch.equal(a, r), k


def test_batch_repeated_calls_and_status():
    print("case batch repeat", flush=True)
    systems, params = _batch(5, "f32", seed=3)
    b = SpectralEwaldBatch(params, [s["N"] for s in systems])
    x = torch.tensor(np.concatenate([s["x"] for s in systems]), device=DEV)
    q = torch.tensor(np.concatenate([s["q"] for s in systems]), device=DEV)
    p1, _, e1 = b(x, q)
    p2, _, e2 = b(x, q)
    assert torch.equal(p1, p2) and torch.equal(e1, e2)   # deterministic
    qn = q.clone()
    qn[0] += 1.0                                         # system 0 (3P) not neutral
    with pytest.raises(_lib.SEError) as e:
        b(x, qn)
    assert e.value.status == _lib.SE_ERR_NONNEUTRAL
    p3, _, _ = b(x, q)
    assert torch.equal(p1, p3)


@pytest.mark.skip(reason="the single cooperative launch with grid-wide barriers between stages hung on the "
                         "GPU (no output for 180 s, GPU still responsive); its cause was not established, so "
                         "that code path was removed and batches run one launch per stage")
def test_batch_single_cooperative_launch():
    pass
