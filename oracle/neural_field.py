"""Discrete neural field: operator, RK4, discrete adjoint, finite differences.

FP64 CPU oracle (test infrastructure).  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the GPU library never does.

What it computes (paper section 2.2, eq. NFODETilde, without forcing):

    u_i'(t) = -u_i + K_i(u),     K_i(u) = sum_j w(|x_i - x_j|) q_j f(u_j),

with q the quadrature weights, the sum over every node j including j = i, and
chordal (Euclidean R^3) distance; or, on the flat domains of the paper's
section 4, the doubly periodic distance of eq. dist (period L in x and in y):
the smallest Euclidean length of x - y + L (i, j, 0) over i, j in {-1, 0, 1}.  Kernels are Mexican hats

    Gaussian:     w(r) = A_e exp(-r^2 / s_e^2) - A_i exp(-r^2 / s_i^2)
    exponential:  w(r) = A_e exp(-r / s_e)     - A_i exp(-r / s_i)

(the paper's eq. winh uses normalised Gaussians; these workloads use the
unnormalised forms), and the firing rate is the sigmoid of eq. firing_rate,
f(u) = 1 / (1 + exp(-beta (u - theta))), with one theta per state.

The time stepper is classical fourth-order Runge-Kutta with a fixed step
(the paper leaves the stepper open apart from its Adams-Bashforth showcase).

The dense sum is written as its definition: a matrix of kernel values in row
panels times the vector q f(u).  No truncation, no reordering beyond the
panel split.  A state array U has shape (B, N): state b is row b.
"""
from __future__ import annotations

import math

import numpy as np

GAUSS_MH = 0
EXP_MH = 1
PANEL_BYTES = 256 << 20


# ------------------------------------------------------------------ pieces


def kernel_w(kind: int, r: np.ndarray, p) -> np.ndarray:
    A_e, s_e, A_i, s_i = p
    if kind == GAUSS_MH:
        return A_e * np.exp(-(r / s_e) ** 2) - A_i * np.exp(-(r / s_i) ** 2)
    if kind == EXP_MH:
        return A_e * np.exp(-r / s_e) - A_i * np.exp(-r / s_i)
    raise ValueError("unknown kernel kind %r" % kind)


def kernel_dw(kind: int, r: np.ndarray, p) -> np.ndarray:
    """Partial derivatives of w(r) w.r.t. (A_e, s_e, A_i, s_i), stacked on axis 0."""
    A_e, s_e, A_i, s_i = p
    if kind == GAUSS_MH:
        ee = np.exp(-(r / s_e) ** 2)
        ei = np.exp(-(r / s_i) ** 2)
        return np.stack([ee, A_e * ee * 2 * r * r / s_e ** 3,
                         -ei, -A_i * ei * 2 * r * r / s_i ** 3])
    if kind == EXP_MH:
        ee = np.exp(-r / s_e)
        ei = np.exp(-r / s_i)
        return np.stack([ee, A_e * ee * r / s_e ** 2, -ei, -A_i * ei * r / s_i ** 2])
    raise ValueError("unknown kernel kind %r" % kind)


def firing(u: np.ndarray, beta: float, theta) -> np.ndarray:
    th = np.asarray(theta, dtype=np.float64).reshape(-1, 1) if np.ndim(u) == 2 else theta
    return 1.0 / (1.0 + np.exp(-beta * (u - th)))


def firing_prime(u: np.ndarray, beta: float, theta) -> np.ndarray:
    f = firing(u, beta, theta)
    return beta * f * (1.0 - f)


def distances(x: np.ndarray, rows, period=None) -> np.ndarray:
    """|x_i - x_j| for i in rows, every j; with a period L, eq. dist: the minimum
    over the nine lattice shifts L (i, j, 0), i, j in {-1, 0, 1}."""
    if not period:
        d = x[rows, None, :] - x[None, :, :]
        return np.sqrt(np.sum(d * d, axis=2))
    dx = x[rows, None, 0] - x[None, :, 0]
    dy = x[rows, None, 1] - x[None, :, 1]
    dz = x[rows, None, 2] - x[None, :, 2]
    sx = [(dx + i * period) ** 2 for i in (-1, 0, 1)]
    sy = [(dy + j * period) ** 2 for j in (-1, 0, 1)]
    best = None
    for a in sx:
        for b in sy:
            best = a + b if best is None else np.minimum(best, a + b)
    return np.sqrt(best + dz * dz)


def _panels(n_rows: int, n_cols: int):
    step = max(1, PANEL_BYTES // (8 * 4 * max(n_cols, 1)))
    for lo in range(0, n_rows, step):
        yield lo, min(n_rows, lo + step)


def kernel_matrix(x: np.ndarray, kind: int, p, rows=None, period=None) -> np.ndarray:
    """w(|x_i - x_j|) for i in rows (default: all), every j."""
    rows = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((rows.size, x.shape[0]))
    for lo, hi in _panels(rows.size, x.shape[0]):
        out[lo:hi] = kernel_w(kind, distances(x, rows[lo:hi], period), p)
    return out


def apply_K(x, q, U, kind, p, beta, theta, rows=None, period=None) -> np.ndarray:
    """K(U) at target rows: sum_j w(|x_i - x_j|) q_j f_b(U[b, j]); shape (B, len(rows)).

    Computed panel by panel from the definition (no stored matrix).
    """
    U = np.atleast_2d(U)
    rows = np.arange(x.shape[0]) if rows is None else np.asarray(rows)
    G = q[None, :] * firing(U, beta, theta)          # (B, N)
    out = np.empty((U.shape[0], rows.size))
    for lo, hi in _panels(rows.size, x.shape[0]):
        Wp = kernel_w(kind, distances(x, rows[lo:hi], period), p)
        out[:, lo:hi] = G @ Wp.T
    return out


class DenseOperator:
    """K with the kernel matrix w_ij stored once (FP64, N x N)."""

    def __init__(self, x, q, kind, p, period=None):
        self.x = np.asarray(x, dtype=np.float64)
        self.q = np.asarray(q, dtype=np.float64)
        self.kind, self.p = kind, tuple(float(v) for v in p)
        self.period = period
        self.w = kernel_matrix(self.x, kind, self.p, period=period)

    @property
    def n(self):
        return self.x.shape[0]

    def K(self, U, beta, theta):
        G = self.q[None, :] * firing(np.atleast_2d(U), beta, theta)
        return G @ self.w.T

    def rhs(self, U, beta, theta):
        return -U + self.K(U, beta, theta)


# ------------------------------------------------------------------ RK4


def rk4_step(op: DenseOperator, u, beta, theta, dt, keep_stages=False):
    v1 = u
    k1 = op.rhs(v1, beta, theta)
    v2 = u + 0.5 * dt * k1
    k2 = op.rhs(v2, beta, theta)
    v3 = u + 0.5 * dt * k2
    k3 = op.rhs(v3, beta, theta)
    v4 = u + dt * k3
    k4 = op.rhs(v4, beta, theta)
    un = u + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    if keep_stages:
        return un, (v1, v2, v3, v4)
    return un


def rk4(op: DenseOperator, u0, beta, theta, dt, steps, save_every=0):
    """Classical RK4 for u' = -u + K(u); returns u(T) (and every save_every-th state)."""
    u = np.array(np.atleast_2d(u0), dtype=np.float64)
    saved = [u.copy()] if save_every else None
    for s in range(steps):
        u = rk4_step(op, u, beta, theta, dt)
        if save_every and (s + 1) % save_every == 0:
            saved.append(u.copy())
    return (u, saved) if save_every else u


# Adams-Bashforth 5 weights of F_n, F_{n-1}, ..., F_{n-4} (times dt).
AB5_WEIGHTS = (1901.0 / 720.0, -2774.0 / 720.0, 2616.0 / 720.0, -1274.0 / 720.0, 251.0 / 720.0)


def ab5(op: DenseOperator, u0, beta, theta, dt, steps):
    """Adams-Bashforth 5, the stepper of the paper's section 5.1 showcase:
    u_{n+1} = u_n + dt sum_k a_k F(u_{n-k}), F(u) = -u + K(u), one operator
    application per step.  The paper does not say how the multistep method is
    started; here the first four steps are classical RK4, and F(u_n) of those
    steps is the first RK4 stage.
    """
    u = np.array(np.atleast_2d(u0), dtype=np.float64)
    hist = []
    for n in range(steps):
        F = op.rhs(u, beta, theta)
        hist = (hist + [F])[-5:]
        if n < 4:
            u = rk4_step(op, u, beta, theta, dt)
        else:
            u = u + dt * sum(a * hist[-1 - k] for k, a in enumerate(AB5_WEIGHTS))
    return u


def syndep_rhs(op: DenseOperator, U, A, beta, theta, tau, beta_d):
    """Neural field with synaptic depression (paper section 5.2, eq. nfsyndep),
    discretised like eq. NFODETilde with the efficacy as a presynaptic field:
      u_i' = -u_i + sum_j w_ij q_j a_j f(u_j),    tau a_i' = 1 - a_i - beta_d a_i f(u_i).
    """
    f = firing(U, beta, theta)
    Ku = (op.q[None, :] * A * f) @ op.w.T
    return -U + Ku, (1.0 - A - beta_d * A * f) / tau


def syndep_rk4(op: DenseOperator, u0, a0, beta, theta, tau, beta_d, dt, steps):
    """Classical RK4 for the coupled (u, a) system of `syndep_rhs`."""
    U = np.array(np.atleast_2d(u0), dtype=np.float64)
    A = np.array(np.atleast_2d(a0), dtype=np.float64)
    for _ in range(steps):
        k1u, k1a = syndep_rhs(op, U, A, beta, theta, tau, beta_d)
        k2u, k2a = syndep_rhs(op, U + 0.5 * dt * k1u, A + 0.5 * dt * k1a, beta, theta, tau, beta_d)
        k3u, k3a = syndep_rhs(op, U + 0.5 * dt * k2u, A + 0.5 * dt * k2a, beta, theta, tau, beta_d)
        k4u, k4a = syndep_rhs(op, U + dt * k3u, A + dt * k3a, beta, theta, tau, beta_d)
        U = U + dt / 6.0 * (k1u + 2 * k2u + 2 * k3u + k4u)
        A = A + dt / 6.0 * (k1a + 2 * k2a + 2 * k3a + k4a)
    return U, A


def rk4_forced(op: DenseOperator, u0, beta, theta, dt, steps, gamma):
    """Classical RK4 for u' = -u + K(u) + gamma(t) (eq. NFODETilde with forcing);
    gamma(n, c) returns the forcing at t_n + c dt for c in (0, 1/2, 1)."""
    u = np.array(np.atleast_2d(u0), dtype=np.float64)
    for n in range(steps):
        g0, gh, g1 = gamma(n, 0.0), gamma(n, 0.5), gamma(n, 1.0)
        k1 = op.rhs(u, beta, theta) + g0
        k2 = op.rhs(u + 0.5 * dt * k1, beta, theta) + gh
        k3 = op.rhs(u + 0.5 * dt * k2, beta, theta) + gh
        k4 = op.rhs(u + dt * k3, beta, theta) + g1
        u = u + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return u


def rk4_rhs_dense(op: DenseOperator, beta, theta):
    """Right-hand side as a plain function of a flat state (for scipy's integrators)."""
    def fun(_t, y):
        return op.rhs(y.reshape(1, -1), beta, theta).ravel()
    return fun


# ------------------------------------------------------------------ adjoint


class ParamOperator(DenseOperator):
    """DenseOperator plus the four kernel-derivative matrices dw/dp."""

    def __init__(self, x, q, kind, p, period=None):
        super().__init__(x, q, kind, p, period)
        r = distances(self.x, np.arange(self.n), period)
        self.dw = kernel_dw(kind, r, self.p)      # (4, N, N)


def loss(uT, target):
    return float(np.sum((uT - target) ** 2))


def adjoint_gradients(op: ParamOperator, u0, beta, theta, dt, steps, target):
    """Discrete adjoint of the RK4 trajectory for L = |u(T) - target|^2.

    Returns (L, dL/du0 (B, N), dL/d(A_e, s_e, A_i, s_i, theta) (5,)), theta a scalar
    shared by all states.  The reverse sweep differentiates each RK4 step as it
    is computed:  with ubar = dL/du_{n+1},
      kbar_1 = kbar_4 = dt/6 ubar,  kbar_2 = kbar_3 = dt/3 ubar,  u_n-bar = ubar,
      for s = 4..1:  vbar_s = J(v_s)^T kbar_s,  u_n-bar += vbar_s,
                     and kbar_{s-1} += c_s dt vbar_s  (c_4 = 1, c_3 = c_2 = 1/2),
    with J(v)^T lam = -lam + (q f'(v)) * (w^T lam).  Parameter cotangents add
    kbar_s^T dG/dp (v_s) at every stage.
    """
    u = np.array(np.atleast_2d(u0), dtype=np.float64)
    traj = [u]
    for _ in range(steps):
        u = rk4_step(op, u, beta, theta, dt)
        traj.append(u)
    L = loss(u, target)
    ubar = 2.0 * (u - target)
    pbar = np.zeros(5)
    coef = {4: 1.0, 3: 0.5, 2: 0.5}
    for n in range(steps - 1, -1, -1):
        _, stages = rk4_step(op, traj[n], beta, theta, dt, keep_stages=True)
        kbar = {1: dt / 6 * ubar, 2: dt / 3 * ubar, 3: dt / 3 * ubar, 4: dt / 6 * ubar}
        un_bar = ubar.copy()
        for s in (4, 3, 2, 1):
            v = stages[s - 1]
            kb = kbar[s]
            f = firing(v, beta, theta)
            fp = firing_prime(v, beta, theta)
            wt_k = kb @ op.w                       # (w^T kbar)_j = sum_i w_ij kbar_i
            vbar = -kb + op.q[None, :] * fp * wt_k
            un_bar += vbar
            g = op.q[None, :] * f
            for m in range(4):
                pbar[m] += float(np.sum(kb * (g @ op.dw[m].T)))
            pbar[4] += float(np.sum(wt_k * op.q[None, :] * (-fp)))
            if s > 1:
                kbar[s - 1] = kbar[s - 1] + coef[s] * dt * vbar
        ubar = un_bar
    return L, ubar, pbar


def _loss_at(x, q, kind, p, u0, beta, theta, dt, steps, target, period=None):
    op = DenseOperator(x, q, kind, p, period)
    return loss(rk4(op, u0, beta, theta, dt, steps), target)


def fd_param_gradients(x, q, kind, p, u0, beta, theta, dt, steps, target, h=1e-4, order=2, period=None):
    """Central finite differences of L in (A_e, s_e, A_i, s_i, theta), absolute step h."""
    base = np.array(list(p) + [theta], dtype=np.float64)
    out = np.zeros(5)
    for m in range(5):
        def L_at(delta):
            v = base.copy()
            v[m] += delta
            return _loss_at(x, q, kind, tuple(v[:4]), u0, beta, v[4], dt, steps, target, period)
        if order == 2:
            out[m] = (L_at(h) - L_at(-h)) / (2 * h)
        else:
            out[m] = (-L_at(2 * h) + 8 * L_at(h) - 8 * L_at(-h) + L_at(-2 * h)) / (12 * h)
    return out


def fd_u0_directional(x, q, kind, p, u0, beta, theta, dt, steps, target, direction,
                      h=1e-4, order=2, period=None):
    op = DenseOperator(x, q, kind, p, period)

    def L_at(delta):
        return loss(rk4(op, u0 + delta * direction, beta, theta, dt, steps), target)
    if order == 2:
        return (L_at(h) - L_at(-h)) / (2 * h)
    return (-L_at(2 * h) + 8 * L_at(h) - 8 * L_at(-h) + L_at(-2 * h)) / (12 * h)


# ------------------------------------------------------------------ metrics


def rel_linf(u, ref) -> np.ndarray:
    """Per-state relative L-infinity error |u - ref|_inf / |ref|_inf."""
    u, ref = np.atleast_2d(u), np.atleast_2d(ref)
    return np.max(np.abs(u - ref), axis=1) / np.max(np.abs(ref), axis=1)
