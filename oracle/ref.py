"""Sequential CPU oracle in plain PyTorch, FP64 (test infrastructure only:
imported by tests, the smoke check and the benchmark's CPU-baseline leg,
never by the product path).

This is the plain definition of what the parallel method computes for the
discretised problem (one implicit-Euler step of the SDE per grid step,
drift/measurement evaluated at the step's right end, R a spectral density):

  * `kalman_filter`  -- covariance-form Kalman filter; the paper identifies
    its backward value-function pass with the Kalman--Bucy filter in
    information form, P = S^{-1}, m = S^{-1} v (Sec. 2.5 and the last
    paragraph of Sec. 4.3).  The log marginal likelihood is accumulated by
    the prediction-error decomposition.
  * `rts_smoother`   -- discrete Rauch--Tung--Striebel smoother; the paper's
    forward trajectory pass is the continuous RTS smoother mean equation
    (Sec. 2.5) and its parallel version (Sec. 4.3, eq. 42).
  * `map_objective`  -- the discretised Onsager--Machlup functional (Sec. 2.1,
    eq. OM) without the divergence term, whose minimiser the smoother mean is.
  * `gauss_newton`   -- iterated Taylor linearisation (Sec. 4.4): linearise
    about the current trajectory, solve the linear-affine problem, repeat.

Everything is a per-step Python loop so that a reader can check it against
the equations by eye; gradients come from torch autograd of these functions.
"""
from __future__ import annotations

import math
import numpy as np
import torch

from . import models

DT = torch.float64


def _step_mats(F, c, L, W, dt):
    """Forward transition of one implicit-Euler step:
    x_k = Phi (x_{k-1} + dt c + w), w ~ N(0, dt Q), Phi = (I - dt F)^{-1}."""
    nx = F.shape[-1]
    Phi = torch.linalg.inv(torch.eye(nx, dtype=DT) - dt * F)
    Q = L @ W @ L.T
    return Phi, Q


def kalman_filter(F, c, L, W, H, r, R, dt, y, m0, P0, dJ=None, deta=None):
    """F [T,nx,nx], c [T,nx], H [T,ny,nx], r [T,ny], dt [T], y [T,ny];
    L, W, R shared by all steps of the segment.  dJ [T,nx,nx], deta [T,nx]
    (optional): one more quadratic cost term 1/2 x^T dJ x - x^T deta on each
    step's right-end state, folded in after the measurement update in
    information form (P <- (P^-1 + dJ)^-1, m <- P (P_old^-1 m_old + deta)).
    Returns m [T+1,nx], P [T+1,nx,nx], predicted mp/Pp [T,...], loglik."""
    T = y.shape[0]
    ny = y.shape[1]
    m, P = m0, P0
    ms, Ps, mps, Pps = [m0], [P0], [], []
    ll = torch.zeros((), dtype=DT)
    for k in range(T):
        Phi, Q = _step_mats(F[k], c[k], L, W, dt[k])
        mp = Phi @ (m + dt[k] * c[k])
        Pp = Phi @ (P + dt[k] * Q) @ Phi.T
        Sg = H[k] @ Pp @ H[k].T + R / dt[k]
        e = y[k] - H[k] @ mp - r[k]
        ll = ll - 0.5 * (ny * math.log(2 * math.pi) + torch.logdet(Sg)
                         + e @ torch.linalg.solve(Sg, e))
        K = Pp @ H[k].T @ torch.linalg.inv(Sg)
        m = mp + K @ e
        P = Pp - K @ Sg @ K.T
        P = 0.5 * (P + P.T)
        if dJ is not None:
            Si = torch.linalg.inv(P)
            P = torch.linalg.inv(Si + dJ[k])
            P = 0.5 * (P + P.T)
            m = P @ (Si @ m + deta[k])
        ms.append(m); Ps.append(P); mps.append(mp); Pps.append(Pp)
    return torch.stack(ms), torch.stack(Ps), torch.stack(mps), torch.stack(Pps), ll


def rts_smoother(F, dt, m, P, mp, Pp):
    """Discrete RTS: G = P_{k-1} Phi_k^T (P^-_k)^{-1},
    xs_{k-1} = m_{k-1} + G (xs_k - m^-_k), Ps_{k-1} = P_{k-1} + G (Ps_k - P^-_k) G^T."""
    T = mp.shape[0]
    nx = m.shape[1]
    xs = [None] * (T + 1)
    Ps = [None] * (T + 1)
    xs[T], Ps[T] = m[T], P[T]
    for k in range(T, 0, -1):
        Phi = torch.linalg.inv(torch.eye(nx, dtype=DT) - dt[k - 1] * F[k - 1])
        G = P[k - 1] @ Phi.T @ torch.linalg.inv(Pp[k - 1])
        xs[k - 1] = m[k - 1] + G @ (xs[k] - mp[k - 1])
        Pk = P[k - 1] + G @ (Ps[k] - Pp[k - 1]) @ G.T
        Ps[k - 1] = 0.5 * (Pk + Pk.T)
    return torch.stack(xs), torch.stack(Ps)


def map_objective(x, F, c, L, W, H, r, R, dt, y, m0, P0):
    """Discretised OM objective (no divergence term) of the linear-affine model:
    1/2 |x0-m0|^2_{P0^-1} + sum_k 1/2 u_k^T (dt W)^{-1} u_k + sum_k dt/2 |y_k - H x_k - r|^2_{R^-1},
    u_k = L^+ (x_k - x_{k-1} - dt (F x_k + c)) the driving-noise increment."""
    d0 = x[0] - m0
    M = 0.5 * d0 @ torch.linalg.solve(P0, d0)
    Lp = torch.linalg.solve(L.T @ L, L.T)
    Winv = torch.linalg.inv(W)
    Rinv = torch.linalg.inv(R)
    for k in range(1, x.shape[0]):
        h = dt[k - 1]
        D = x[k] - x[k - 1] - h * (F[k - 1] @ x[k] + c[k - 1])
        u = Lp @ D
        eps = y[k - 1] - H[k - 1] @ x[k] - r[k - 1]
        M = M + 0.5 * u @ Winv @ u / h + 0.5 * h * eps @ Rinv @ eps
    return M


def map_objective_nonlinear(model, theta, x, dt, y, m0, P0, nx):
    """Same objective with the nonlinear drift and measurement evaluated at
    the right-end state (the function Gauss--Newton minimises)."""
    T = x.shape[0] - 1
    f, hx = models.drift_torch(model, theta, x[1:], nx)
    _, _, L, W, _, _, R = models.terms_torch(model, theta, x[1:], nx)
    d0 = x[0] - m0
    M = 0.5 * d0 @ torch.linalg.solve(P0, d0)
    Lp = torch.linalg.solve(L.T @ L, L.T)
    Winv = torch.linalg.inv(W)
    Rinv = torch.linalg.inv(R)
    for k in range(1, T + 1):
        h = dt[k - 1]
        u = Lp @ (x[k] - x[k - 1] - h * f[k - 1])
        eps = y[k - 1] - hx[k - 1]
        if model == "ct":
            eps = torch.stack([eps[0], models.wrap_angle(eps[1])])
        M = M + 0.5 * u @ Winv @ u / h + 0.5 * h * eps @ Rinv @ eps
    return M


def divergence_expansion(model, theta, xbar, dt, nx):
    """Second-order Taylor expansion about xbar [T, nx] of each step's term
    1/2 dt_k div f(x_k) of the Onsager--Machlup objective (Sec. 2.1, eq. OM),
    written as 1/2 x^T dJ x - x^T deta + const (the form of an element's J and
    eta): dJ = 1/2 dt Hess, deta = -1/2 dt (grad - Hess xbar), gradient and
    Hessian of div f by autograd."""
    dJ, deta = [], []
    for k in range(xbar.shape[0]):
        xk = xbar[k].detach()
        fn = lambda x: models.divergence_torch(model, theta.detach(), x[None], nx)[0]
        g = torch.autograd.functional.jacobian(fn, xk)
        Hs = torch.autograd.functional.hessian(fn, xk)
        dJ.append(0.5 * dt[k] * Hs)
        deta.append(-0.5 * dt[k] * (g - Hs @ xk))
    return torch.stack(dJ), torch.stack(deta)


def om_objective(model, theta, x, dt, y, m0, P0, nx):
    """The discretised Onsager--Machlup objective with its divergence term:
    map_objective_nonlinear + sum_k 1/2 dt_k div f(x_k)."""
    div = models.divergence_torch(model, theta, x[1:], nx)
    return map_objective_nonlinear(model, theta, x, dt, y, m0, P0, nx) + 0.5 * (dt * div).sum()


def smooth_segment(model, theta, xbar, dt, y, m0, P0, nx, lin=None, om_div=False):
    """One linear-affine solve about xbar [T+1, nx] (states).  Returns a dict
    with filter m, P, smoother xs, Ps, loglik and mstar = M_d(xs).  For the
    model "linear" the matrices come from `lin` (torch tensors, per step).
    With om_div, the divergence term of eq. OM enters by its second-order
    expansion about xbar (a Newton step on it), and mstar includes the term
    at xs (loglik is then not meaningful)."""
    if lin is not None:
        F, c, L, W, H, r, R = (lin[k] for k in ("F", "c", "L", "W", "H", "r", "R"))
    else:
        F, c, L, W, H, r, R = models.terms_torch(model, theta, xbar[1:], nx, y)
    dJ = deta = None
    if om_div:
        dJ, deta = divergence_expansion(model, theta, xbar[1:], dt, nx)
    m, P, mp, Pp, ll = kalman_filter(F, c, L, W, H, r, R, dt, y, m0, P0, dJ, deta)
    xs, Ps = rts_smoother(F, dt, m, P, mp, Pp)
    M = map_objective(xs, F, c, L, W, H, r, R, dt, y, m0, P0)
    if om_div:
        M = M + 0.5 * (dt * models.divergence_torch(model, theta, xs[1:], nx)).sum()
    return dict(m=m, P=P, xs=xs, Ps=Ps, loglik=ll, mstar=M)


def gauss_newton(model, theta, dt, y, m0, P0, nx, n_iter, xbar0=None, om_div=False):
    """Iterated linearisation (Sec. 4.4).  xbar^(0) = m0 at every state unless
    given.  Returns the list of iterates [xbar^(1), ..., xbar^(n_iter)] and the
    outputs of the last linear solve (whose linearisation point is the
    iterate before it, held fixed).  om_div: see smooth_segment."""
    T = y.shape[0]
    xbar = m0.expand(T + 1, nx).clone() if xbar0 is None else xbar0
    its = []
    out = None
    for _ in range(n_iter):
        out = smooth_segment(model, theta, xbar.detach(), dt, y, m0, P0, nx, om_div=om_div)
        out["xbar"] = xbar.detach()
        xbar = out["xs"]
        its.append(xbar.detach())
    return its, out


def workload_segment(wl, s):
    """Torch FP64 views of segment s of a `workloads.Workload`."""
    st = wl.seg_steps(s)
    lin = None
    if wl.lin is not None:
        lin = {k: torch.tensor(np.asarray(v[st] if k in ("F", "c", "H", "r") else v), dtype=DT)
               for k, v in wl.lin.items()}
    return dict(lin=lin, theta=torch.tensor(wl.theta[s], dtype=DT),
                dt=torch.tensor(wl.dt[st], dtype=DT),
                y=torch.tensor(wl.y[:, st].T.copy(), dtype=DT),
                m0=torch.tensor(wl.m0[s], dtype=DT),
                P0=torch.tensor(wl.P0[s], dtype=DT))


def gradients(model, nx, seg, xbar):
    """d loglik / d theta and d mstar / d theta by autograd of the plain
    definitions above, linearisation point xbar [T+1, nx] held fixed."""
    th = seg["theta"].clone().requires_grad_(True)
    out = smooth_segment(model, th, xbar.detach(), seg["dt"], seg["y"], seg["m0"], seg["P0"], nx)
    gl, = torch.autograd.grad(out["loglik"], th, retain_graph=True)
    gm, = torch.autograd.grad(out["mstar"], th)
    return gl, gm, out


def trajectory_vjp(model, nx, seg, xbar, w):
    """d (sum_k w_k . xs_k) / d theta by autograd of the plain definitions
    above (w [T+1, nx] a fixed cotangent of the MAP trajectory), linearisation
    point xbar [T+1, nx] held fixed."""
    th = seg["theta"].clone().requires_grad_(True)
    out = smooth_segment(model, th, xbar.detach(), seg["dt"], seg["y"], seg["m0"], seg["P0"], nx)
    g, = torch.autograd.grad((out["xs"] * w).sum(), th)
    return g
