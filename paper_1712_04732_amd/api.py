"""PyTorch face of the library: plans over torch device memory and streams,
and the hand-written adjoint behind torch.autograd.Function.

Every computation is a call of the HIP library through the C ABI; torch only
provides device tensors and the current stream.
"""
from __future__ import annotations

import torch

from . import _lib as L

_WINDOWS = {"gaussian": L.SE_WIN_GAUSSIAN, "pkb": L.SE_WIN_PKB, "es": L.SE_WIN_ES}
_PRECS = {"f64": L.SE_F64, "f32": L.SE_F32}


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _workspace(nbytes):
    """A torch-owned device block for a plan's work buffers (the caching
    allocator aligns blocks to 512 bytes, the library needs 256)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def _check_out(out, N, dtype, dev, e_shape):
    """Caller-supplied outputs (phi, force, energy): each None or a contiguous
    tensor on the input's device with shape (N,), (N, 3), e_shape and dtype
    dtype, dtype, float64.  The kernels write N rows without bounds checks, so
    a mismatch is an error here."""
    for t, shape, dt in zip(out, ((N,), (N, 3), e_shape), (dtype, dtype, torch.float64)):
        if t is None:
            continue
        if (not isinstance(t, torch.Tensor) or tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous()
                or t.device != dev):
            raise ValueError("output tensors must be contiguous, on the input's device, with the plan's "
                             f"shapes and dtypes: expected {shape} {dt}")


class SpectralEwald:
    """A plan for one system size class: periodicity D, box L, Ewald xi, grid M,
    window support P.  Parameters left as None follow the paper's rules
    (Section 6); s and n_l need either explicit values or Q and tol.
    force_method 1 differentiates the gathering window, 2 multiplies the
    scaling step by i k (Section 7.2); with 2 the autograd functions receive
    method 2's gradient, an approximation of the discrete energy's gradient
    to the method's accuracy.  My, Mz make the periodic cell rectangular at
    h = L/M: a triply periodic box L x My h x Mz h (D = 3), or a doubly
    periodic cell L x My h with z free (D = 2, My only).

    Call it with positions x (N,3) and charges q (N,) on the GPU.
    """

    def __init__(self, D, L_box, xi, M, P, *, window="pkb", prec="f64", n_max=1 << 20,
                 Q=None, tol=None, shape=None, nu=None, lam=None, s0=None, s=None, n_l=None,
                 tile=0, force_method=1, deriv_fit=False, My=0, Mz=0):
        if not torch.cuda.is_available():
            raise RuntimeError("SpectralEwald needs a HIP device")
        L.load()
        w = _WINDOWS[window]
        pr = _PRECS[prec]
        if Q is not None and tol is not None:
            p = L.se_params_default(D, L_box, xi, M, P, w, Q, tol, pr)
        else:
            p = L.se_params()
            p.D, p.L, p.xi, p.M, p.P, p.window, p.prec = D, L_box, xi, M, P, w, pr
            p.n_l = -1
        if shape is not None:
            p.shape = shape
        if nu is not None:
            p.nu = nu
        if lam is not None:
            p.lambda_ = lam
        if s0 is not None:
            p.s0 = s0
        if s is not None:
            p.s = s
        if n_l is not None:
            p.n_l = n_l
        p.tile = tile
        p.force_method = force_method
        p.deriv_fit = 1 if deriv_fit else 0
        # rectangular periodic cell L x My h (x Mz h in 3P), h = L / M; 0: square
        p.My, p.Mz = int(My), int(Mz)
        self.params = p
        self.n_max = int(n_max)
        self.prec = prec
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        self.D, self.L, self.xi = D, L_box, xi
        self._plan = L.se_plan_create(p, self.n_max, _stream())
        self.info = L.se_plan_get_info(self._plan)
        self._bind()

    @property
    def box(self):
        """The box sides: (L, L, L) for a cube, (L, My h, Mz h) at h = L / M
        for a rectangular one."""
        p = self.params
        h = p.L / p.M
        return (p.L, p.My * h if p.My > 0 else p.L, p.Mz * h if p.Mz > 0 else p.L)

    def _bind(self):
        self.workspace = _workspace(L.se_plan_workspace_size(self._plan))
        L.se_plan_set_workspace(self._plan, self.workspace.data_ptr(), self.workspace.numel())

    @classmethod
    def from_params(cls, p, n_max):
        """A plan from a filled se_params (for example one returned by
        autotune)."""
        self = cls.__new__(cls)
        if not torch.cuda.is_available():
            raise RuntimeError("SpectralEwald needs a HIP device")
        L.load()
        self.params = p
        self.n_max = int(n_max)
        self.prec = "f64" if p.prec == L.SE_F64 else "f32"
        self.dtype = torch.float64 if p.prec == L.SE_F64 else torch.float32
        self.D, self.L, self.xi = p.D, p.L, p.xi
        self._plan = L.se_plan_create(p, self.n_max, _stream())
        self.info = L.se_plan_get_info(self._plan)
        self._bind()
        return self

    def autotune(self, x, q, allow_nonneutral=False):
        """Schedule knobs timed on the input (x, q); returns a new plan with
        the chosen knobs and the tuner's report."""
        x, q = _device_pair(x, q)
        flags = (L.SE_IN_F32 if x.dtype == torch.float32 else 0) | (
            L.SE_ALLOW_NONNEUTRAL if allow_nonneutral else 0)
        p, rep = L.se_autotune(self.params, x.shape[0], x.data_ptr(), q.data_ptr(), flags, _stream())
        return SpectralEwald.from_params(p, self.n_max), rep

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            try:
                L.se_plan_destroy(plan)
            except Exception:
                pass
            self._plan = None

    def profile(self, reset=True):
        """Per-launch-site timings of the evaluations made with profile=True."""
        return L.se_plan_profile(self._plan, _stream(), reset)

    def evaluate(self, x, q, *, phi=True, force=True, energy=True, add_self=False,
                 out_grad=False, check=True, allow_nonneutral=False, profile=False, out=None):
        """One evaluation of Algorithm 4.  Returns (phi, force_or_grad, energy);
        entries not requested are None."""
        if x.dim() != 2 or x.shape[1] != 3 or q.dim() != 1 or q.shape[0] != x.shape[0]:
            raise ValueError("x must be (N,3) and q (N,)")
        if x.dtype != q.dtype or x.dtype not in (torch.float32, torch.float64):
            raise ValueError("x and q must share dtype float32 or float64")
        if not (x.is_cuda and q.is_cuda):
            raise ValueError("x and q must be device tensors")
        x = x.contiguous()
        q = q.contiguous()
        N = x.shape[0]
        dev = x.device
        if out is not None:
            out_phi, out_f, out_e = out
            _check_out(out, N, self.dtype, dev, ())
        else:
            out_phi = torch.empty(N, dtype=self.dtype, device=dev) if phi else None
            out_f = torch.empty((N, 3), dtype=self.dtype, device=dev) if force else None
            out_e = torch.empty((), dtype=torch.float64, device=dev) if energy else None
        phi, force, energy = out_phi is not None, out_f is not None, out_e is not None
        flags = 0
        if x.dtype == torch.float32:
            flags |= L.SE_IN_F32
        if add_self:
            flags |= L.SE_ADD_SELF
        if out_grad:
            flags |= L.SE_OUT_GRAD
        if check:
            flags |= L.SE_SYNC_CHECK
        if allow_nonneutral:
            flags |= L.SE_ALLOW_NONNEUTRAL
        if profile:
            flags |= L.SE_PROFILE
        st = L.se_eval(self._plan, N, x.data_ptr(), q.data_ptr(),
                       out_phi.data_ptr() if phi else 0, out_f.data_ptr() if force else 0,
                       out_e.data_ptr() if energy else 0, flags, _stream())
        if st != L.SE_OK:
            raise L.SEError(st, "se_eval")
        return out_phi, out_f, out_e

    __call__ = evaluate


def _device_pair(x, q):
    if x.dim() != 2 or x.shape[1] != 3 or q.dim() != 1 or q.shape[0] != x.shape[0]:
        raise ValueError("x must be (N,3) and q (N,)")
    if x.dtype != q.dtype or x.dtype not in (torch.float32, torch.float64):
        raise ValueError("x and q must share dtype float32 or float64")
    if not (x.is_cuda and q.is_cuda):
        raise ValueError("x and q must be device tensors")
    return x.contiguous(), q.contiguous()


def _params(D, L_box, xi, M, P, window="pkb", prec="f64", Q=None, tol=None, s=None, n_l=None, tile=0):
    w = _WINDOWS[window]
    pr = _PRECS[prec]
    if Q is not None and tol is not None:
        p = L.se_params_default(D, L_box, xi, M, P, w, Q, tol, pr)
    else:
        p = L.se_params()
        p.D, p.L, p.xi, p.M, p.P, p.window, p.prec = D, L_box, xi, M, P, w, pr
        p.n_l = -1
    if s is not None:
        p.s = s
    if n_l is not None:
        p.n_l = n_l
    p.tile = tile
    return p


def params_for_tolerance(D, L_box, xi, Q, tol_rel, P=8, window="pkb", prec="f32"):
    """Grid size and AFT parameters for a relative tolerance at a given
    window support P (Section 6 rules, P chosen by the caller)."""
    return L.se_params_for_tolerance(D, L_box, xi, Q, tol_rel, P, _WINDOWS[window], _PRECS[prec])


def params_recipe(D, L_box, xi, Q, tol_rel, window="pkb", prec="f64"):
    """The whole Section 6 recipe: M and P from the tolerance, with the
    error-pollution remedy (M + 5 %, P + 4)."""
    return L.se_params_recipe(D, L_box, xi, Q, tol_rel, _WINDOWS[window], _PRECS[prec])


class SpectralEwaldBatch:
    """Many independent systems evaluated together: one launch per stage of
    the path over the work items of all systems.

    params: list of se_params (one per system, same P, window and precision);
    N: particles per system.  Inputs and outputs are concatenated in system
    order."""

    def __init__(self, params, N):
        if not torch.cuda.is_available():
            raise RuntimeError("SpectralEwaldBatch needs a HIP device")
        L.load()
        self.params = list(params)
        self.N = [int(n) for n in N]
        self.n_sys = len(self.N)
        self.total = sum(self.N)
        self.dtype = torch.float64 if self.params[0].prec == L.SE_F64 else torch.float32
        self._plan = L.se_batch_plan_create(self.params, self.N, _stream())
        self.workspace = _workspace(L.se_batch_plan_workspace_size(self._plan))
        L.se_batch_plan_set_workspace(self._plan, self.workspace.data_ptr(), self.workspace.numel())

    @classmethod
    def tuned(cls, params, N, x, q, allow_nonneutral=False):
        """A batch plan whose schedule knobs the autotuner chose on the input
        (x, q); returns (plan, report)."""
        if not torch.cuda.is_available():
            raise RuntimeError("SpectralEwaldBatch needs a HIP device")
        total = sum(int(n) for n in N)
        if x.shape != (total, 3) or q.shape != (total,):
            raise ValueError("x must be (sum N, 3) and q (sum N,)")
        if x.dtype != q.dtype or x.dtype not in (torch.float32, torch.float64) or not (x.is_cuda and q.is_cuda):
            raise ValueError("x and q must be device tensors of one dtype, float32 or float64")
        x, q = x.contiguous(), q.contiguous()
        flags = (L.SE_IN_F32 if x.dtype == torch.float32 else 0) | (
            L.SE_ALLOW_NONNEUTRAL if allow_nonneutral else 0)
        tp, rep = L.se_batch_autotune(list(params), N, x.data_ptr(), q.data_ptr(), flags, _stream())
        return cls(tp, N), rep

    def info(self, sys):
        return L.se_batch_plan_get_info(self._plan, sys)[0]

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            try:
                L.se_batch_plan_destroy(plan)
            except Exception:
                pass
            self._plan = None

    def profile(self, reset=True):
        return L.se_batch_plan_profile(self._plan, _stream(), reset)

    def evaluate(self, x, q, *, phi=True, force=True, energy=True, add_self=False, out_grad=False,
                 check=True, allow_nonneutral=False, profile=False, out=None):
        if x.shape != (self.total, 3) or q.shape != (self.total,):
            raise ValueError("x must be (sum N, 3) and q (sum N,)")
        if x.dtype != q.dtype or x.dtype not in (torch.float32, torch.float64) or not (x.is_cuda and q.is_cuda):
            raise ValueError("x and q must be device tensors of one dtype, float32 or float64")
        x = x.contiguous()
        q = q.contiguous()
        dev = x.device
        if out is not None:
            out_phi, out_f, out_e = out
            _check_out(out, self.total, self.dtype, dev, (self.n_sys,))
        else:
            out_phi = torch.empty(self.total, dtype=self.dtype, device=dev) if phi else None
            out_f = torch.empty((self.total, 3), dtype=self.dtype, device=dev) if force else None
            out_e = torch.empty(self.n_sys, dtype=torch.float64, device=dev) if energy else None
        flags = 0
        if x.dtype == torch.float32:
            flags |= L.SE_IN_F32
        if add_self:
            flags |= L.SE_ADD_SELF
        if out_grad:
            flags |= L.SE_OUT_GRAD
        if check:
            flags |= L.SE_SYNC_CHECK
        if allow_nonneutral:
            flags |= L.SE_ALLOW_NONNEUTRAL
        if profile:
            flags |= L.SE_PROFILE
        st = L.se_eval_batch(self._plan, x.data_ptr(), q.data_ptr(),
                             out_phi.data_ptr() if out_phi is not None else 0,
                             out_f.data_ptr() if out_f is not None else 0,
                             out_e.data_ptr() if out_e is not None else 0, flags, _stream())
        if st != L.SE_OK:
            raise L.SEError(st, "se_eval_batch")
        return out_phi, out_f, out_e

    __call__ = evaluate


def _energy_backward(gE, q, phi, grad, prec, needs_x, needs_q):
    """dE/dx = gE q grad phi and dE/dq = gE phi, computed by se_energy_vjp."""
    N = q.shape[0]
    gx = torch.empty((N, 3), dtype=q.dtype, device=q.device) if needs_x else None
    gq = torch.empty_like(q) if needs_q else None
    gE = gE.to(device=q.device, dtype=torch.float64).contiguous()
    st = L.se_energy_vjp(N, prec, gE.data_ptr(), q.data_ptr(), phi.data_ptr(), grad.data_ptr(),
                         gx.data_ptr() if gx is not None else 0, gq.data_ptr() if gq is not None else 0,
                         L.SE_IN_F32 if q.dtype == torch.float32 else 0, _stream())
    if st != L.SE_OK:
        raise L.SEError(st, "se_energy_vjp")
    return gx, gq


class SEEnergy(torch.autograd.Function):
    """E = 1/2 sum_m q_m phi_m (k-space part, plus the self energy when
    add_self).  Backward (se_energy_vjp): dE/dq = phi, dE/dx_m = q_m grad
    phi(x_m), the gradient of the gathering window (Eq. force-method-1)."""

    @staticmethod
    def forward(ctx, x, q, plan: SpectralEwald, add_self: bool = False):
        x, q = _device_pair(x.detach(), q.detach())
        phi, grad, E = plan.evaluate(x, q, out_grad=True, add_self=add_self)
        ctx.save_for_backward(q, phi, grad)
        ctx.prec = plan.params.prec
        return E

    @staticmethod
    def backward(ctx, gE):
        q, phi, grad = ctx.saved_tensors
        gx, gq = _energy_backward(gE, q, phi, grad, ctx.prec, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gx, gq, None, None


class EwaldEnergy(torch.autograd.Function):
    """Total electrostatic energy of Eq. (potential_split),
    E = 1/2 sum_m q_m (phi^F + phi^R + phi^self)_m: the k-space part by the
    SpectralEwald plan (with the self term), the real-space part by the
    RealSpace plan accumulated into the same outputs.  Backward
    (se_energy_vjp): dE/dq = phi, dE/dx_m = q_m grad phi(x_m)."""

    @staticmethod
    def forward(ctx, x, q, kplan: SpectralEwald, rplan: "RealSpace"):
        xd, qd = _device_pair(x.detach(), q.detach())
        out = kplan.evaluate(xd, qd, out_grad=True, add_self=True)
        phi, grad, E = rplan.evaluate(xd, qd, out_grad=True, accumulate=True, out=out)
        ctx.save_for_backward(qd, phi, grad)
        ctx.prec = kplan.params.prec
        return E

    @staticmethod
    def backward(ctx, gE):
        q, phi, grad = ctx.saved_tensors
        gx, gq = _energy_backward(gE, q, phi, grad, ctx.prec, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gx, gq, None, None


class SEPotential(torch.autograd.Function):
    """phi = A(x) q.  The discrete operator A (spread, scale, gather with one
    window) is symmetric, so for a cotangent g (se_eval_vjp):
        dL/dq   = A g
        dL/dx_m = g_m grad phi(x_m) + q_m grad (A g)(x_m)."""

    @staticmethod
    def forward(ctx, x, q, plan: SpectralEwald, add_self: bool = False):
        x, q = _device_pair(x.detach(), q.detach())
        phi, grad, _ = plan.evaluate(x, q, out_grad=True, energy=False, add_self=add_self)
        ctx.save_for_backward(x, q, grad)
        ctx.plan = plan
        ctx.add_self = add_self
        return phi

    @staticmethod
    def backward(ctx, g):
        x, q, grad = ctx.saved_tensors
        plan = ctx.plan
        N = x.shape[0]
        g = g.to(x.dtype).contiguous()
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gq = torch.empty_like(q) if ctx.needs_input_grad[1] else None
        flags = (L.SE_IN_F32 if x.dtype == torch.float32 else 0) | (L.SE_ADD_SELF if ctx.add_self else 0)
        st = L.se_eval_vjp(plan._plan, N, x.data_ptr(), q.data_ptr(), g.data_ptr(), grad.data_ptr(),
                           gx.data_ptr() if gx is not None else 0, gq.data_ptr() if gq is not None else 0,
                           flags, _stream())
        if st != L.SE_OK:
            raise L.SEError(st, "se_eval_vjp")
        return gx, gq, None, None


class RealSpace:
    """The real-space sum of the Ewald split, Eq. (real_space_ewald), with
    cutoff rc, on the GPU (cell list in the HIP library).  Adds to a k-space
    result of SpectralEwald (accumulate=True) to give the full potential of
    Eq. (potential_split).  L_box is the side of a cube, or the three sides
    of a rectangular box (SpectralEwald(..., My, Mz).box: free directions
    extend over their side)."""

    def __init__(self, D, L_box, xi, rc, *, prec="f64", n_max=1 << 20, cells_per_rc=0):
        if not torch.cuda.is_available():
            raise RuntimeError("RealSpace needs a HIP device")
        L.load()
        self.D, self.xi, self.rc = D, xi, rc
        self.prec = prec
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        self.n_max = int(n_max)
        if isinstance(L_box, (tuple, list)):
            if len(L_box) != 3:
                raise ValueError("a rectangular box takes three sides")
            self.L = self.box = tuple(float(v) for v in L_box)
            self._plan = L.se_rs_plan_create_box(D, self.box, xi, rc, self.n_max, _PRECS[prec], cells_per_rc,
                                                 _stream())
            _, _, self.device_bytes = L.se_rs_get_info(self._plan)
            self.cells, self.span = L.se_rs_cells_box(self.box, rc, self.n_max, cells_per_rc)
        else:
            self.L = L_box
            self.box = (float(L_box),) * 3
            self._plan = L.se_rs_plan_create(D, L_box, xi, rc, self.n_max, _PRECS[prec], cells_per_rc, _stream())
            self.cells, self.span, self.device_bytes = L.se_rs_get_info(self._plan)
        self.workspace = _workspace(L.se_rs_workspace_size(self._plan))
        L.se_rs_set_workspace(self._plan, self.workspace.data_ptr(), self.workspace.numel())

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            try:
                L.se_rs_plan_destroy(plan)
            except Exception:
                pass
            self._plan = None

    def profile(self, reset=True):
        """HIP-event times of the evaluations made with profile=True."""
        return L.se_rs_plan_profile(self._plan, _stream(), reset)

    def evaluate(self, x, q, *, phi=True, force=True, energy=True, out_grad=False, accumulate=False,
                 check=True, profile=False, out=None):
        """Returns (phi^R, force_or_grad, E^R); with accumulate=True the
        results are added into out = (phi, force, energy)."""
        x, q = _device_pair(x, q)
        N = x.shape[0]
        dev = x.device
        if out is not None:
            out_phi, out_f, out_e = out
        elif accumulate:
            raise ValueError("accumulate=True needs out")
        else:
            out_phi = torch.empty(N, dtype=self.dtype, device=dev) if phi else None
            out_f = torch.empty((N, 3), dtype=self.dtype, device=dev) if force else None
            out_e = torch.empty((), dtype=torch.float64, device=dev) if energy else None
        _check_out((out_phi, out_f, out_e), N, self.dtype, dev, ())
        flags = (L.SE_IN_F32 if x.dtype == torch.float32 else 0) | (L.SE_OUT_GRAD if out_grad else 0) | (
            L.SE_ACCUMULATE if accumulate else 0) | (L.SE_SYNC_CHECK if check else 0) | (
            L.SE_PROFILE if profile else 0)
        st = L.se_rs_eval(self._plan, N, x.data_ptr(), q.data_ptr(),
                          out_phi.data_ptr() if out_phi is not None else 0,
                          out_f.data_ptr() if out_f is not None else 0,
                          out_e.data_ptr() if out_e is not None else 0, flags, _stream())
        if st != L.SE_OK:
            raise L.SEError(st, "se_rs_eval")
        return out_phi, out_f, out_e

    __call__ = evaluate
