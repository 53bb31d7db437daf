"""Caller-owned workspaces and the device adjoint entries of the C ABI.

Every work buffer of an evaluation lies in a workspace the caller binds (torch
tensors in the Python layer); plans own only their tables.  These tests bind,
rebind and share workspaces and check that results are unchanged bit for bit,
and that the adjoint entries (se_energy_vjp, se_eval_vjp) equal the chain rule
written out with torch on the CPU in float64.
"""
import ctypes

import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1712_04732_amd import (RealSpace, SpectralEwald, SpectralEwaldBatch, _lib,  # noqa: E402
                                  params_for_tolerance)

DEV = torch.device("cuda:0")


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _inputs(N, seed, dtype=torch.float64, kind="pm1"):
    x, q = wl.system(N, 1.0, seed, kind)
    return torch.tensor(x, dtype=dtype, device=DEV), torch.tensor(q, dtype=dtype, device=DEV)


def test_evaluation_needs_a_bound_workspace():
    print("case workspace unbound", flush=True)
    plan = SpectralEwald(3, 1.0, 8.0, 32, 8, prec="f64", n_max=256)
    x, q = _inputs(256, 11)
    nbytes = _lib.se_plan_workspace_size(plan._plan)
    assert nbytes == plan.info.workspace_bytes > 0
    _lib.se_plan_set_workspace(plan._plan, 0, 0)         # unbind
    st = _lib.se_eval(plan._plan, 256, x.data_ptr(), q.data_ptr(), 0, 0, 0, 0, _stream())
    assert st == _lib.SE_ERR_WORKSPACE
    lib = _lib.load()
    ws = torch.empty(nbytes + 512, dtype=torch.uint8, device=DEV)
    assert lib.se_plan_set_workspace(plan._plan, ctypes.c_void_p(ws.data_ptr()), nbytes - 1) == _lib.SE_ERR_WORKSPACE
    assert lib.se_plan_set_workspace(plan._plan, ctypes.c_void_p(ws.data_ptr() + 8), nbytes) == _lib.SE_ERR_WORKSPACE
    assert lib.se_plan_set_workspace(plan._plan, ctypes.c_void_p(ws.data_ptr() + 256), nbytes) == _lib.SE_OK
    phi, g, E = plan(x, q, out_grad=True)
    torch.cuda.synchronize()
    assert torch.isfinite(phi).all() and torch.isfinite(g).all()


@pytest.mark.parametrize("D", [3, 2, 1, 0])
def test_rebinding_and_sharing_keep_results(D):
    """A plan rebound to another workspace, and two plans taking turns on one
    workspace, compute the same numbers bit for bit."""
    print(f"case workspace rebinding D={D}", flush=True)
    N = 3000
    kw = dict(s=2.0, n_l=3) if D in (1, 2) else {}
    a = SpectralEwald(D, 1.0, 9.0, 30, 8, prec="f64", n_max=N, **kw)
    b = SpectralEwald(D, 1.0, 7.0, 24, 6, prec="f64", n_max=N, **kw)
    x, q = _inputs(N, 40 + D)
    ra = [t.clone() for t in a(x, q, out_grad=True)]
    rb = [t.clone() for t in b(x, q, out_grad=True)]
    shared = torch.empty(max(a.info.workspace_bytes, b.info.workspace_bytes), dtype=torch.uint8, device=DEV)
    shared.fill_(0xAB)   # contents need no initialisation
    for p in (a, b):
        _lib.se_plan_set_workspace(p._plan, shared.data_ptr(), shared.numel())
    for _ in range(2):
        for p, ref in ((a, ra), (b, rb)):
            out = p(x, q, out_grad=True)
            for u, v in zip(out, ref):
                assert torch.equal(u, v)


def test_batch_and_real_space_rebinding():
    print("case workspace batch and real space", flush=True)
    params, Ns, xs, qs = [], [], [], []
    for k, D in enumerate((3, 2, 1, 0)):
        n = 300 + 50 * k
        x, q = wl.system(n, 1.0, 70 + k, "pm1")
        params.append(params_for_tolerance(D, 1.0, wl.batch_xi(n, 1.0), float(n), 1e-7, 8, "pkb", "f32"))
        Ns.append(n)
        xs.append(x)
        qs.append(q)
    batch = SpectralEwaldBatch(params, Ns)
    bx = torch.tensor(np.concatenate(xs), dtype=torch.float32, device=DEV)
    bq = torch.tensor(np.concatenate(qs), dtype=torch.float32, device=DEV)
    ref = [t.clone() for t in batch(bx, bq)]
    ws = torch.full((_lib.se_batch_plan_workspace_size(batch._plan) + 1024,), 7, dtype=torch.uint8, device=DEV)
    _lib.se_batch_plan_set_workspace(batch._plan, ws.data_ptr() + 512, ws.numel() - 512)
    for u, v in zip(batch(bx, bq), ref):
        assert torch.equal(u, v)
    _lib.se_batch_plan_set_workspace(batch._plan, 0, 0)
    st = _lib.se_eval_batch(batch._plan, bx.data_ptr(), bq.data_ptr(), 0, 0, 0, _lib.SE_IN_F32, _stream())
    assert st == _lib.SE_ERR_WORKSPACE

    rs = RealSpace(3, 1.0, 12.0, 0.25, prec="f64", n_max=500)
    x, q = _inputs(500, 90)
    rref = [t.clone() for t in rs(x, q, out_grad=True)]
    ws2 = torch.empty(_lib.se_rs_workspace_size(rs._plan), dtype=torch.uint8, device=DEV)
    _lib.se_rs_set_workspace(rs._plan, ws2.data_ptr(), ws2.numel())
    for u, v in zip(rs(x, q, out_grad=True), rref):
        assert torch.equal(u, v)


@pytest.mark.parametrize("prec,dt", [("f64", torch.float64), ("f64", torch.float32), ("f32", torch.float32)])
def test_energy_vjp_is_the_chain_rule(prec, dt):
    """se_energy_vjp writes gE q grad phi and gE phi (FP64 arithmetic, input
    precision out); compared with the same products in float64 on the CPU."""
    print(f"case energy vjp {prec} {dt}", flush=True)
    N = 1000
    plan = SpectralEwald(3, 1.0, 8.0, 32, 8, prec=prec, n_max=N)
    x, q = _inputs(N, 123, dt)
    phi, grad, _ = plan(x, q, out_grad=True)
    gE = torch.tensor(-1.75, dtype=torch.float64, device=DEV)
    gx = torch.empty_like(x)
    gq = torch.empty_like(q)
    st = _lib.se_energy_vjp(N, plan.params.prec, gE.data_ptr(), q.data_ptr(), phi.data_ptr(), grad.data_ptr(),
                            gx.data_ptr(), gq.data_ptr(), _lib.SE_IN_F32 if dt == torch.float32 else 0, _stream())
    assert st == _lib.SE_OK
    torch.cuda.synchronize()
    qc, pc, gc = q.cpu().double(), phi.cpu().double(), grad.cpu().double()
    assert torch.equal(gx.cpu(), (-1.75 * qc[:, None] * gc).to(dt))
    assert torch.equal(gq.cpu(), (-1.75 * pc).to(dt))


@pytest.mark.parametrize("D", [3, 0])
def test_potential_vjp_entry_matches_two_evaluations(D):
    """se_eval_vjp against its definition: A g and grad(A g) from a plain
    evaluation with the cotangent as charges, combined on the CPU in float64."""
    print(f"case potential vjp entry D={D}", flush=True)
    N = 800
    plan = SpectralEwald(D, 1.0, 8.0, 28, 8, prec="f64", n_max=N)
    x, q = _inputs(N, 300 + D, kind="uniform")
    g = torch.tensor(np.random.default_rng(4).standard_normal(N), device=DEV)
    _, grad, _ = plan(x, q, out_grad=True, energy=False, add_self=True)
    ag, agrad, _ = plan(x, g, out_grad=True, energy=False, add_self=True, allow_nonneutral=True)
    gx = torch.empty_like(x)
    gq = torch.empty_like(q)
    st = _lib.se_eval_vjp(plan._plan, N, x.data_ptr(), q.data_ptr(), g.data_ptr(), grad.data_ptr(),
                          gx.data_ptr(), gq.data_ptr(), _lib.SE_ADD_SELF | _lib.SE_SYNC_CHECK, _stream())
    assert st == _lib.SE_OK
    torch.cuda.synchronize()
    assert torch.equal(gq, ag)
    want = g.cpu()[:, None] * grad.cpu() + q.cpu()[:, None] * agrad.cpu()
    # the device may contract the product and the sum into one fused multiply-add
    assert torch.allclose(gx.cpu(), want, rtol=1e-15, atol=1e-15 * float(want.abs().max()))
    # grad_q alone (no saved gradient needed)
    gq2 = torch.empty_like(q)
    st = _lib.se_eval_vjp(plan._plan, N, x.data_ptr(), q.data_ptr(), g.data_ptr(), 0, 0, gq2.data_ptr(),
                          _lib.SE_ADD_SELF, _stream())
    assert st == _lib.SE_OK
    torch.cuda.synchronize()
    assert torch.equal(gq2, ag)
