"""Model terms for the oracle (test infrastructure only; never imported by the
product path).

For a state-space model of the paper's form (Sec. 2.1, eq. statespace)

    dx/dt = f(x) + L w,   y = h(x) + v,   w, v white with spectral densities W, R,

the linear-affine model of Sec. 2.4 (eq. linear-statespace) used at one
Gauss--Newton iteration is the first-order Taylor expansion about a nominal
state xbar (Sec. 4.4):

    F = df/dx(xbar),  c = f(xbar) - F xbar,  H = dh/dx(xbar),  r = h(xbar) - H xbar.

Every term is evaluated at the right end of its grid step, i.e. at the state
x_k the step leads to.  Two implementations are given: torch (differentiable
in theta, for gradient truth by autograd) and numpy (vectorised over steps,
feeding the C oracle).

Parameter vectors:
  cv        (gamma, q, r): F = [[0, I], [0, -gamma I]], c = 0, L = [0; I], W = q I,
                           H = [I, 0], r = 0, R = r I          (nx = 2d, ny = nw = d)
  vdp       (mu, q, r):    f = (x2, mu (1 - x1^2) x2 - x1), L = I, W = q I,
                           h = x1, R = r                        (nx = 2, ny = 1, nw = 2)
  lorenz63  (sigma, rho, beta, q, r): f = (sigma (x2 - x1), x1 (rho - x3) - x2,
                           x1 x2 - beta x3), L = I, W = q I, h = x, R = r I  (nx = ny = nw = 3)
  ct        (sv, sw, r1, r2): coordinated turn of Sec. 5.2, x = (xi, zeta, dxi, dzeta, omega),
                           f = (dxi, dzeta, -omega dzeta, omega dxi, 0),
                           L = [[0,0,0],[0,0,0],[sv,0,0],[0,sv,0],[0,0,sw]], W = I,
                           h = (sqrt(xi^2 + zeta^2), atan2(zeta, xi)), R = diag(r1, r2)
                           (nx = 5, ny = 2, nw = 3).  The bearing residual y - h is taken
                           modulo 2 pi into [-pi, pi) (`wrap_angle`); with y given, the
                           returned r is shifted by the multiple of 2 pi that does this for
                           y - r (H xbar has no bearing part: H_bearing xbar = 0).

The paper writes the bearing as arctan(zeta / xi); atan2 is the same on the
half-plane xi > 0 and continues it to every direction.
"""
from __future__ import annotations

import numpy as np
import torch


TWO_PI = 2.0 * np.pi
INV_2PI = 1.0 / TWO_PI


def wrap_angle(e):
    """e modulo 2 pi into [-pi, pi): e - 2 pi floor(e / (2 pi) + 1/2)."""
    if torch.is_tensor(e):
        return e - TWO_PI * torch.floor(e * INV_2PI + 0.5)
    return e - TWO_PI * np.floor(e * INV_2PI + 0.5)


def dims(model: str, nx: int):
    if model == "cv":
        return nx, nx // 2, nx // 2
    if model == "vdp":
        return 2, 1, 2
    if model == "lorenz63":
        return 3, 3, 3
    if model == "ct":
        return 5, 2, 3
    raise ValueError(model)


def _ct_L(sv, sw, like):
    L = like.new_zeros(5, 3) if torch.is_tensor(like) else np.zeros((5, 3))
    L[2, 0] = sv
    L[3, 1] = sv
    L[4, 2] = sw
    return L


# ----------------------------------------------------------------------------- torch

def terms_torch(model: str, theta: torch.Tensor, xbar: torch.Tensor, nx: int, y=None):
    """theta [n_theta]; xbar [T, nx] (the right-end state of each step); y [T, ny]
    (only used by ct, for the bearing wrap).
    Returns F [T,nx,nx], c [T,nx], L [nx,nw], W [nw,nw], H [T,ny,nx], r [T,ny], R [ny,ny]."""
    T = xbar.shape[0]
    dt_ = theta.dtype
    if model == "ct":
        sv, sw, r1, r2 = theta[0], theta[1], theta[2], theta[3]
        xi, ze, dxi, dze, om = (xbar[:, i] for i in range(5))
        zero = torch.zeros_like(xi)
        one = torch.ones_like(xi)
        F = torch.stack([torch.stack([zero, zero, one, zero, zero], 1),
                         torch.stack([zero, zero, zero, one, zero], 1),
                         torch.stack([zero, zero, zero, -om, -dze], 1),
                         torch.stack([zero, zero, om, zero, dxi], 1),
                         torch.stack([zero, zero, zero, zero, zero], 1)], 1)
        f = torch.stack([dxi, dze, -om * dze, om * dxi, zero], 1)
        c = f - torch.einsum("kij,kj->ki", F, xbar)
        rho2 = xi * xi + ze * ze
        rho = torch.sqrt(rho2)
        H = torch.stack([torch.stack([xi / rho, ze / rho, zero, zero, zero], 1),
                         torch.stack([-ze / rho2, xi / rho2, zero, zero, zero], 1)], 1)
        hx = torch.stack([rho, torch.atan2(ze, xi)], 1)
        r = hx - torch.einsum("kij,kj->ki", H, xbar)
        if y is not None:
            r = torch.stack([r[:, 0], y[:, 1] - wrap_angle(y[:, 1] - r[:, 1])], 1)
        L = _ct_L(sv, sw, theta)
        R = torch.diag(torch.stack([r1, r2]))
        return F, c, L, torch.eye(3, dtype=dt_), H, r, R
    if model == "cv":
        d = nx // 2
        g, q, rr = theta[0], theta[1], theta[2]
        I = torch.eye(d, dtype=dt_)
        Z = torch.zeros(d, d, dtype=dt_)
        F = torch.cat([torch.cat([Z, I], 1), torch.cat([Z, -g * I], 1)], 0)
        F = F.expand(T, nx, nx)
        c = torch.zeros(T, nx, dtype=dt_)
        L = torch.cat([Z, I], 0)
        W = q * I
        H = torch.cat([I, Z], 1).expand(T, d, nx)
        r = torch.zeros(T, d, dtype=dt_)
        R = rr * I
        return F, c, L, W, H, r, R
    if model == "vdp":
        mu, q, rr = theta[0], theta[1], theta[2]
        x1, x2 = xbar[:, 0], xbar[:, 1]
        zero = torch.zeros_like(x1)
        one = torch.ones_like(x1)
        F = torch.stack([torch.stack([zero, one], 1),
                         torch.stack([-2.0 * mu * x1 * x2 - 1.0, mu * (1.0 - x1 * x1)], 1)], 1)
        f = torch.stack([x2, mu * (1.0 - x1 * x1) * x2 - x1], 1)
        c = f - torch.einsum("kij,kj->ki", F, xbar)
        L = torch.eye(2, dtype=dt_)
        W = q * torch.eye(2, dtype=dt_)
        H = torch.tensor([[1.0, 0.0]], dtype=dt_).expand(T, 1, 2)
        r = torch.zeros(T, 1, dtype=dt_)
        R = rr.reshape(1, 1)
        return F, c, L, W, H, r, R
    if model == "lorenz63":
        sg, rho, be, q, rr = theta[0], theta[1], theta[2], theta[3], theta[4]
        x1, x2, x3 = xbar[:, 0], xbar[:, 1], xbar[:, 2]
        one = torch.ones_like(x1)
        F = torch.stack([torch.stack([-sg * one, sg * one, 0.0 * one], 1),
                         torch.stack([rho - x3, -one, -x1], 1),
                         torch.stack([x2, x1, -be * one], 1)], 1)
        f = torch.stack([sg * (x2 - x1), x1 * (rho - x3) - x2, x1 * x2 - be * x3], 1)
        c = f - torch.einsum("kij,kj->ki", F, xbar)
        L = torch.eye(3, dtype=dt_)
        W = q * torch.eye(3, dtype=dt_)
        H = torch.eye(3, dtype=dt_).expand(T, 3, 3)
        r = torch.zeros(T, 3, dtype=dt_)
        R = rr * torch.eye(3, dtype=dt_)
        return F, c, L, W, H, r, R
    raise ValueError(model)


def drift_torch(model: str, theta: torch.Tensor, x: torch.Tensor, nx: int):
    """The nonlinear drift f(x) and measurement h(x), x [T, nx]."""
    if model == "ct":
        xi, ze, dxi, dze, om = (x[:, i] for i in range(5))
        f = torch.stack([dxi, dze, -om * dze, om * dxi, torch.zeros_like(xi)], 1)
        return f, torch.stack([torch.sqrt(xi * xi + ze * ze), torch.atan2(ze, xi)], 1)
    if model == "cv":
        d = nx // 2
        g = theta[0]
        f = torch.cat([x[:, d:], -g * x[:, d:]], 1)
        return f, x[:, :d]
    if model == "vdp":
        mu = theta[0]
        x1, x2 = x[:, 0], x[:, 1]
        return torch.stack([x2, mu * (1.0 - x1 * x1) * x2 - x1], 1), x[:, :1]
    if model == "lorenz63":
        sg, rho, be = theta[0], theta[1], theta[2]
        x1, x2, x3 = x[:, 0], x[:, 1], x[:, 2]
        return torch.stack([sg * (x2 - x1), x1 * (rho - x3) - x2, x1 * x2 - be * x3], 1), x
    raise ValueError(model)


def divergence_torch(model: str, theta: torch.Tensor, x: torch.Tensor, nx: int):
    """div f(x) = trace of the drift's Jacobian, the divergence term of the
    Onsager--Machlup functional (Sec. 2.1, eq. OM), x [T, nx] -> [T]."""
    T = x.shape[0]
    if model == "cv":
        return -(nx // 2) * theta[0] * torch.ones(T, dtype=x.dtype)
    if model == "vdp":
        return theta[0] * (1.0 - x[:, 0] * x[:, 0])
    if model == "lorenz63":
        return -(theta[0] + 1.0 + theta[2]) * torch.ones(T, dtype=x.dtype)
    if model == "ct":
        return torch.zeros(T, dtype=x.dtype)
    raise ValueError(model)


# ----------------------------------------------------------------------------- numpy

def terms_numpy(model: str, theta: np.ndarray, xbar: np.ndarray, nx: int, y=None):
    """Same terms as `terms_torch`, vectorised: theta [n_theta] (one segment),
    xbar [T, nx], y [T, ny] (ct only).  Per-step arrays have a leading T axis."""
    T = xbar.shape[0]
    if model == "ct":
        sv, sw, r1, r2 = theta
        xi, ze, dxi, dze, om = (xbar[:, i] for i in range(5))
        F = np.zeros((T, 5, 5))
        F[:, 0, 2] = 1.0
        F[:, 1, 3] = 1.0
        F[:, 2, 3] = -om
        F[:, 2, 4] = -dze
        F[:, 3, 2] = om
        F[:, 3, 4] = dxi
        f = np.stack([dxi, dze, -om * dze, om * dxi, np.zeros(T)], 1)
        c = f - np.einsum("kij,kj->ki", F, xbar)
        rho2 = xi * xi + ze * ze
        rho = np.sqrt(rho2)
        H = np.zeros((T, 2, 5))
        H[:, 0, 0] = xi / rho
        H[:, 0, 1] = ze / rho
        H[:, 1, 0] = -ze / rho2
        H[:, 1, 1] = xi / rho2
        hx = np.stack([rho, np.arctan2(ze, xi)], 1)
        r = hx - np.einsum("kij,kj->ki", H, xbar)
        if y is not None:
            r[:, 1] = y[:, 1] - wrap_angle(y[:, 1] - r[:, 1])
        return F, c, _ct_L(sv, sw, xbar), np.eye(3), H, r, np.diag([r1, r2])
    if model == "cv":
        d = nx // 2
        g, q, rr = theta
        F = np.zeros((nx, nx))
        F[:d, d:] = np.eye(d)
        F[d:, d:] = -g * np.eye(d)
        L = np.zeros((nx, d))
        L[d:, :] = np.eye(d)
        H = np.zeros((d, nx))
        H[:, :d] = np.eye(d)
        return (np.broadcast_to(F, (T, nx, nx)), np.zeros((T, nx)), L, q * np.eye(d),
                np.broadcast_to(H, (T, d, nx)), np.zeros((T, d)), rr * np.eye(d))
    if model == "vdp":
        mu, q, rr = theta
        x1, x2 = xbar[:, 0], xbar[:, 1]
        F = np.zeros((T, 2, 2))
        F[:, 0, 1] = 1.0
        F[:, 1, 0] = -2.0 * mu * x1 * x2 - 1.0
        F[:, 1, 1] = mu * (1.0 - x1 * x1)
        f = np.stack([x2, mu * (1.0 - x1 * x1) * x2 - x1], 1)
        c = f - np.einsum("kij,kj->ki", F, xbar)
        H = np.broadcast_to(np.array([[1.0, 0.0]]), (T, 1, 2))
        return F, c, np.eye(2), q * np.eye(2), H, np.zeros((T, 1)), np.array([[rr]])
    if model == "lorenz63":
        sg, rho, be, q, rr = theta
        x1, x2, x3 = xbar[:, 0], xbar[:, 1], xbar[:, 2]
        F = np.zeros((T, 3, 3))
        F[:, 0, 0] = -sg
        F[:, 0, 1] = sg
        F[:, 1, 0] = rho - x3
        F[:, 1, 1] = -1.0
        F[:, 1, 2] = -x1
        F[:, 2, 0] = x2
        F[:, 2, 1] = x1
        F[:, 2, 2] = -be
        f = np.stack([sg * (x2 - x1), x1 * (rho - x3) - x2, x1 * x2 - be * x3], 1)
        c = f - np.einsum("kij,kj->ki", F, xbar)
        H = np.broadcast_to(np.eye(3), (T, 3, 3))
        return F, c, np.eye(3), q * np.eye(3), H, np.zeros((T, 3)), rr * np.eye(3)
    raise ValueError(model)
