"""Thin torch-facing wrapper over the C ABI (argument marshalling only).

Every computation runs in libnfr.so.  PyTorch provides device memory and the
stream; tensors are passed as raw device pointers.  States are (B, N) float64
CUDA tensors: state b is row b, i.e. the state-major N x B layout of the ABI.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int, c_void_p

import torch

from . import _lib as L


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _dev_buffer(nbytes: int, device, stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """256-byte aligned device bytes.  With `stream`, the block is allocated while
    that stream is current, so torch's caching allocator orders its reuse after
    the work the library enqueues there (the library runs on the context's
    stream, which need not be the caller's current stream)."""
    if stream is not None:
        with torch.cuda.stream(stream):
            return _dev_buffer(nbytes, device)
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 1)]


def kernel_struct(kind: int, A_e: float, s_e: float, A_i: float, s_i: float) -> L.NfrKernel:
    return L.NfrKernel(int(kind), float(A_e), float(s_e), float(A_i), float(s_i))


class Firing:
    """Sigmoid firing rate; `theta` is a float or a per-state CUDA float64 tensor."""

    def __init__(self, beta: float, theta):
        self.beta = float(beta)
        if isinstance(theta, torch.Tensor):
            self.theta_t = theta.to(torch.float64).contiguous()
            self.theta = 0.0
        else:
            self.theta_t = None
            self.theta = float(theta)

    def struct(self, device) -> L.NfrFiring:
        tp = None
        if self.theta_t is not None:
            if self.theta_t.device != device:
                self.theta_t = self.theta_t.to(device)
            tp = self.theta_t.data_ptr()
        return L.NfrFiring(self.beta, self.theta, tp)


class Context:
    """A device and the stream every call of the library is enqueued on."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = c_void_p()
        L.check(L.lib().nfr_context_create(device, c_void_p(self.stream.cuda_stream), byref(h)))
        self.handle = h

    def order_after_caller(self) -> None:
        """Makes the context's stream wait for the caller's current stream, so that
        inputs the caller produced (or copied with .to()/.contiguous()) are complete
        before the library reads them.  Results are complete on `self.stream`;
        a caller on another stream waits for it before reading them."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    @property
    def arch(self) -> str:
        return L.lib().nfr_context_arch(self.handle).decode()

    def close(self):
        if self.handle:
            L.lib().nfr_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Packed node set: xyz (N, 3) and q (N,) float64 CUDA tensors.  With
    period L > 0 the (x, y) plane is doubly periodic (nfr_problem_create_periodic)."""

    def __init__(self, ctx: Context, xyz: torch.Tensor, q: torch.Tensor, period: float = 0.0):
        if xyz.dim() != 2 or xyz.shape[1] != 3 or q.shape != (xyz.shape[0],):
            raise ValueError("xyz must be (N, 3) and q (N,)")
        self.ctx = ctx
        self.n = int(xyz.shape[0])
        xyz = xyz.to(ctx.device, torch.float64).contiguous()
        q = q.to(ctx.device, torch.float64).contiguous()
        nbytes = L.lib().nfr_problem_bytes(self.n)
        if nbytes == 0:
            raise ValueError("unsupported problem size %d" % self.n)
        self.pack = _dev_buffer(nbytes, ctx.device, ctx.stream)
        h = c_void_p()
        ctx.order_after_caller()
        with torch.cuda.stream(ctx.stream):
            L.check(L.lib().nfr_problem_create_periodic(ctx.handle, self.n, xyz.data_ptr(), q.data_ptr(),
                                                        float(period), self.pack.data_ptr(), nbytes, byref(h)))
        self._keep = (xyz, q)            # the pack kernel reads them asynchronously
        self.handle = h
        self.npad = int(L.lib().nfr_problem_npad(h))
        self.period = float(L.lib().nfr_problem_period(h))

    def close(self):
        if self.handle:
            L.lib().nfr_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ W form

    def w_build(self, kernel: L.NfrKernel, form: int) -> torch.Tensor:
        nbytes = L.lib().nfr_w_bytes(self.n, form)
        if nbytes == 0:
            raise ValueError("form %d has no W matrix" % form)
        W = _dev_buffer(nbytes, self.ctx.device, self.ctx.stream)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_w_build(self.handle, byref(kernel), form, W.data_ptr(), nbytes))
        return W

    # ------------------------------------------------------------ operator

    def _check_state(self, u: torch.Tensor) -> int:
        if u.dtype != torch.float64 or u.dim() != 2 or u.shape[1] != self.n or not u.is_contiguous():
            raise ValueError("state must be a contiguous (B, N) float64 tensor")
        if u.device != self.ctx.device:
            raise ValueError("state is on %s, context on %s" % (u.device, self.ctx.device))
        return int(u.shape[0])

    def apply(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, form: int = L.FORM_ONTHEFLY_FP32,
              W: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
        B = self._check_state(u)
        if out is None:
            with torch.cuda.stream(self.ctx.stream):
                out = torch.empty_like(u)
        y = out
        ws_bytes = L.lib().nfr_apply_workspace_size(self.handle, B, form)
        ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_apply(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), y.data_ptr(), form,
                                  _ptr(W), ws.data_ptr(), ws_bytes))
        self._last_ws = ws
        return y

    def apply_noalloc(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, out: torch.Tensor,
                      form: int = L.FORM_ONTHEFLY_FP32, W: torch.Tensor | None = None) -> torch.Tensor:
        """nfr_apply_noalloc: the operator into the caller's `out` with the library's
        fixed device scratch (no allocation by the library or by this method)."""
        B = self._check_state(u)
        if out.shape != u.shape or out.dtype != torch.float64 or not out.is_contiguous() or out.device != u.device:
            raise ValueError("out must be a contiguous float64 tensor shaped like u, on its device")
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_apply_noalloc(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), out.data_ptr(),
                                          form, _ptr(W)))
        return out

    def integrate(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, dt: float, steps: int,
                  form: int = L.FORM_ONTHEFLY_FP32, W: torch.Tensor | None = None, ckpt_every: int = 0,
                  use_graph: bool = False, ws: torch.Tensor | None = None):
        """Advances u in place by `steps` RK4 steps; returns checkpoints (K, B, N) or None."""
        B = self._check_state(u)
        ws_bytes = L.lib().nfr_integrate_workspace_size(self.handle, B, form)
        if ws is None or ws.numel() < ws_bytes:
            ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        ck = None
        if ckpt_every:
            with torch.cuda.stream(self.ctx.stream):
                ck = torch.empty((1 + steps // ckpt_every, B, self.n), dtype=torch.float64, device=self.ctx.device)
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_integrate(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), float(dt), int(steps),
                                      form, _ptr(W), _ptr(ck), int(ckpt_every), int(bool(use_graph)),
                                      ws.data_ptr(), ws_bytes))
        self._last_ws = ws
        return ck

    def integrate_forced(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, dt: float, steps: int,
                         forcing: torch.Tensor, form: int = L.FORM_ONTHEFLY_FP32, W: torch.Tensor | None = None):
        """RK4 with forcing; forcing is (steps, 3, B, N) float64: gamma at t_n, t_n + dt/2, t_n + dt."""
        B = self._check_state(u)
        if tuple(forcing.shape) != (steps, 3, B, self.n) or forcing.dtype != torch.float64:
            raise ValueError("forcing must be a (steps, 3, B, N) float64 tensor")
        forcing = forcing.to(self.ctx.device).contiguous()
        ws_bytes = L.lib().nfr_integrate_workspace_size(self.handle, B, form)
        ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_integrate_forced(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), float(dt),
                                             int(steps), forcing.data_ptr(), form, _ptr(W), ws.data_ptr(), ws_bytes))
        self._last_ws = (ws, forcing)

    def integrate_ab5(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, dt: float, steps: int,
                      form: int = L.FORM_ONTHEFLY_FP32, W: torch.Tensor | None = None, ws: torch.Tensor | None = None):
        """Advances u in place by `steps` Adams-Bashforth 5 steps (RK4 start-up)."""
        B = self._check_state(u)
        ws_bytes = L.lib().nfr_integrate_ab5_workspace_size(self.handle, B, form)
        if ws is None or ws.numel() < ws_bytes:
            ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_integrate_ab5(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), float(dt),
                                          int(steps), form, _ptr(W), ws.data_ptr(), ws_bytes))
        self._last_ws = ws

    def integrate_syndep(self, kernel: L.NfrKernel, firing: Firing, u: torch.Tensor, a: torch.Tensor, tau: float,
                         beta_d: float, dt: float, steps: int, ws: torch.Tensor | None = None):
        """Advances (u, a) in place: neural field with synaptic depression, RK4."""
        B = self._check_state(u)
        if self._check_state(a) != B:
            raise ValueError("u and a must have the same shape")
        ws_bytes = L.lib().nfr_integrate_syndep_workspace_size(self.handle, B)
        if ws is None or ws.numel() < ws_bytes:
            ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_integrate_syndep(self.handle, byref(kernel), byref(fs), B, u.data_ptr(), a.data_ptr(),
                                             float(tau), float(beta_d), float(dt), int(steps), ws.data_ptr(),
                                             ws_bytes))
        self._last_ws = ws

    def adjoint(self, kernel: L.NfrKernel, firing: Firing, ckpt: torch.Tensor, ckpt_every: int, steps: int,
                dt: float, ubarT: torch.Tensor):
        """Discrete-adjoint gradients of L(u(T)) for a single state: (dL/du0 (N,), dL/dp (5,) float64)."""
        if ubarT.shape != (self.n,) and ubarT.shape != (1, self.n):
            raise ValueError("ubarT must hold N values")
        ubarT = ubarT.reshape(self.n).to(self.ctx.device, torch.float64).contiguous()
        ckpt = ckpt.to(self.ctx.device, torch.float64).contiguous()
        need = 1 + steps // ckpt_every
        if ckpt.numel() < need * self.n:
            raise ValueError("ckpt holds %d states, %d needed" % (ckpt.numel() // self.n, need))
        ws_bytes = L.lib().nfr_adjoint_workspace_size(self.handle, int(steps), int(ckpt_every))
        ws = _dev_buffer(ws_bytes, self.ctx.device, self.ctx.stream)
        with torch.cuda.stream(self.ctx.stream):
            ubar0 = torch.empty(self.n, dtype=torch.float64, device=self.ctx.device)
        pbar = (c_double * 5)()
        fs = firing.struct(self.ctx.device)
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_adjoint(self.handle, byref(kernel), byref(fs), ckpt.data_ptr(), int(ckpt_every),
                                    int(steps), float(dt), ubarT.data_ptr(), ubar0.data_ptr(), pbar,
                                    ws.data_ptr(), ws_bytes))
        return ubar0, torch.tensor(list(pbar), dtype=torch.float64)

    def far_blocks(self, kernel: L.NfrKernel) -> tuple[int, int]:
        """nfr_far_blocks: (blocks of the fused BF16 form that skip the steep exponential,
        all blocks) for this kernel; synchronises the context stream."""
        nbytes = L.lib().nfr_far_blocks_workspace_size(self.handle)
        ws = _dev_buffer(nbytes, self.ctx.device, self.ctx.stream)
        far, tot = ctypes.c_int64(), ctypes.c_int64()
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_far_blocks(self.handle, byref(kernel), ws.data_ptr(), nbytes, byref(far), byref(tot)))
        return int(far.value), int(tot.value)

    def integrate_workspace(self, B: int, form: int) -> torch.Tensor:
        return _dev_buffer(L.lib().nfr_integrate_workspace_size(self.handle, B, form), self.ctx.device, self.ctx.stream)


class Batch:
    """Problems of one context time-stepped together (nfr_batch_*): one persistent
    pair-sum launch and one combine launch per RK4 stage for all of them."""

    def __init__(self, ctx: Context, problems, kernels, firings, Bs):
        P = len(problems)
        if not (P == len(kernels) == len(firings) == len(Bs)) or P == 0:
            raise ValueError("problems, kernels, firings and Bs must have the same non-zero length")
        self.ctx, self.problems, self.Bs = ctx, list(problems), [int(b) for b in Bs]
        self._firings = list(firings)
        ph = (c_void_p * P)(*[p.handle.value for p in problems])
        ks = (L.NfrKernel * P)(*kernels)
        fs = (L.NfrFiring * P)(*[f.struct(ctx.device) for f in firings])
        bs = (c_int * P)(*self.Bs)
        h = c_void_p()
        L.check(L.lib().nfr_batch_create(ctx.handle, P, ph, ks, fs, bs, byref(h)))
        self.handle = h

    def _states(self, states):
        if len(states) != len(self.problems):
            raise ValueError("one state tensor per problem")
        for p, u, B in zip(self.problems, states, self.Bs):
            if p._check_state(u) != B:
                raise ValueError("state of problem with B=%d has %d rows" % (B, u.shape[0]))
        return (c_void_p * len(states))(*[u.data_ptr() for u in states])

    def workspace(self) -> torch.Tensor:
        return _dev_buffer(L.lib().nfr_batch_workspace_size(self.handle), self.ctx.device, self.ctx.stream)

    @property
    def config(self):
        c, w = ctypes.c_int64(), c_int()
        L.check(L.lib().nfr_batch_get_config(self.handle, byref(c), byref(w)))
        return int(c.value), int(w.value)

    @config.setter
    def config(self, cw):
        L.check(L.lib().nfr_batch_set_config(self.handle, int(cw[0]), int(cw[1])))

    def tune(self, states, ws: torch.Tensor | None = None) -> float:
        ws = self.workspace() if ws is None else ws
        best = c_double()
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_batch_tune(self.handle, self._states(states), ws.data_ptr(), ws.numel(), byref(best)))
        return best.value

    def integrate(self, states, dt: float, steps: int, use_graph: bool = False, ws: torch.Tensor | None = None):
        ptrs = self._states(states)
        ws = self.workspace() if ws is None else ws
        self.ctx.order_after_caller()
        L.check(L.lib().nfr_batch_integrate(self.handle, ptrs, float(dt), int(steps), int(bool(use_graph)),
                                            ws.data_ptr(), ws.numel()))

    def close(self):
        if self.handle:
            L.lib().nfr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(ctx: Context, cache_path: str | None = None, n_max: int = 65536, B_max: int = 64) -> None:
    """Autotunes the multi-state on-the-fly pair sum (nfr_tune); results apply process-wide."""
    ws_bytes = L.lib().nfr_tune_workspace_size(int(n_max), int(B_max))
    if ws_bytes == 0:
        raise ValueError("unsupported tuning sizes n_max=%d, B_max=%d" % (n_max, B_max))
    ws = _dev_buffer(ws_bytes, ctx.device, ctx.stream)
    path = cache_path.encode() if cache_path else None
    L.check(L.lib().nfr_tune(ctx.handle, path, int(n_max), int(B_max), ws.data_ptr(), ws_bytes))


def tune_load(cache_path: str) -> None:
    L.check(L.lib().nfr_tune_load(cache_path.encode()))


def quad_weights(ctx: Context, xyz: torch.Tensor, normals: torch.Tensor, tris, projection, k: int = 32,
                 details: bool = False):
    """Surface quadrature weights q (N,) float64 on the GPU (nfr_quad_weights).

    xyz, normals: (N, 3) float64 (moved to the context's device); tris: (M, 3)
    integer array-like (host), oriented outward.  projection: L.PROJ_PLANES,
    L.PROJ_ORIGIN or L.PROJ_ORTHOGONAL (a bool is read as "star-shaped":
    True -> PROJ_ORIGIN, False -> PROJ_PLANES).  With details=True also
    returns the stencils (M, k) int32 and projection points (M, 3) float64.
    """
    import numpy as np
    tri = np.ascontiguousarray(np.asarray(tris), dtype=np.int32)
    if tri.ndim != 2 or tri.shape[1] != 3:
        raise ValueError("tris must be (M, 3)")
    xyz = xyz.to(ctx.device, torch.float64).contiguous()
    normals = normals.to(ctx.device, torch.float64).contiguous()
    n, m = int(xyz.shape[0]), int(tri.shape[0])
    ws_bytes = L.lib().nfr_quad_workspace_size(n, m, k)
    if ws_bytes == 0:
        raise ValueError("unsupported sizes n=%d, triangles=%d, k=%d" % (n, m, k))
    ws = _dev_buffer(ws_bytes, ctx.device, ctx.stream)
    ctx.order_after_caller()
    with torch.cuda.stream(ctx.stream):
        q = torch.empty(n, dtype=torch.float64, device=ctx.device)
        st = torch.empty((m, k), dtype=torch.int32, device=ctx.device) if details else None
        pj = torch.empty((m, 3), dtype=torch.float64, device=ctx.device) if details else None
        L.check(L.lib().nfr_quad_weights(ctx.handle, n, xyz.data_ptr(), normals.data_ptr(), m,
                                         tri.ctypes.data_as(c_void_p), int(projection), int(k),
                                         q.data_ptr(), _ptr(st), _ptr(pj), ws.data_ptr(), ws_bytes))
    if details:
        return q, st, pj
    return q


class NeuralFieldRK4(torch.autograd.Function):
    """u(T) = RK4^steps(u0; A_e, s_e, A_i, s_i, theta) on a packed problem, single state.

    forward: nfr_integrate (on-the-fly FP32 pair sums, FP64 state) keeping
    checkpoints every `ckpt_every` steps; backward: nfr_adjoint.  On a context
    with its own stream both replay captured HIP graphs.  `params` is
    a CPU float64 tensor (A_e, s_e, A_i, s_i, theta); its gradient is returned
    on the CPU.
    """

    @staticmethod
    def forward(ctx, u0, params, problem, kind, beta, dt, steps, ckpt_every):
        p = [float(v) for v in params.detach().cpu().tolist()]
        k = kernel_struct(kind, *p[:4])
        f = Firing(beta, p[4])
        u = u0.detach().reshape(1, problem.n).to(torch.float64).clone().contiguous()
        graphs = problem.ctx.stream.cuda_stream != 0      # the null stream cannot be captured
        ck = problem.integrate(k, f, u, dt, steps, form=L.FORM_ONTHEFLY_FP32, ckpt_every=ckpt_every,
                               use_graph=graphs)
        ctx.problem, ctx.k, ctx.f = problem, k, f
        ctx.dt, ctx.steps, ctx.every = dt, steps, ckpt_every
        ctx.save_for_backward(ck)
        ctx.u0_shape = u0.shape
        return u.reshape(u0.shape)

    @staticmethod
    def backward(ctx, grad_u):
        (ck,) = ctx.saved_tensors
        gu0, gp = ctx.problem.adjoint(ctx.k, ctx.f, ck, ctx.every, ctx.steps, ctx.dt, grad_u.reshape(-1))
        return gu0.reshape(ctx.u0_shape), gp, None, None, None, None, None, None
