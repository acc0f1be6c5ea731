"""Brute-force dense references that pin the oracle (tests only).

Nothing here shares code with `oracle/`: the discretised model (one
implicit-Euler step per grid step, per-sample measurement covariance R/dt)
is written out once more as a joint Gaussian over all states and
measurements, and as a stacked least-squares problem, and solved with dense
linear algebra.
"""
from __future__ import annotations

import numpy as np


def step_terms(wl, s, xbar=None):
    """Model terms per step of segment s as dense numpy arrays (test-side copy)."""
    T = wl.seg_off[s + 1] - wl.seg_off[s]
    st = wl.seg_steps(s)
    nx, ny, nw = wl.nx, wl.ny, wl.nw
    if wl.model == "linear":
        lin = wl.lin
        return (lin["F"][st], lin["c"][st], lin["L"], lin["W"], lin["H"][st], lin["r"][st],
                lin["R"])
    th = wl.theta[s]
    if wl.model == "cv":
        d = nx // 2
        g, q, rr = th
        F = np.zeros((nx, nx)); F[:d, d:] = np.eye(d); F[d:, d:] = -g * np.eye(d)
        L = np.vstack([np.zeros((d, d)), np.eye(d)])
        H = np.hstack([np.eye(d), np.zeros((d, d))])
        return (np.repeat(F[None], T, 0), np.zeros((T, nx)), L, q * np.eye(d),
                np.repeat(H[None], T, 0), np.zeros((T, d)), rr * np.eye(d))
    xb = xbar[:, st.start + s + 1: st.stop + s + 1].T
    if wl.model == "vdp":
        mu, q, rr = th
        F = np.zeros((T, 2, 2))
        c = np.zeros((T, 2))
        for k in range(T):
            a, b = xb[k]
            F[k] = [[0.0, 1.0], [-2 * mu * a * b - 1.0, mu * (1 - a * a)]]
            c[k] = np.array([b, mu * (1 - a * a) * b - a]) - F[k] @ xb[k]
        return (F, c, np.eye(2), q * np.eye(2), np.repeat(np.array([[[1.0, 0.0]]]), T, 0),
                np.zeros((T, 1)), np.array([[rr]]))
    if wl.model == "lorenz63":
        sg, rho, be, q, rr = th
        F = np.zeros((T, 3, 3))
        c = np.zeros((T, 3))
        for k in range(T):
            a, b, e = xb[k]
            F[k] = [[-sg, sg, 0.0], [rho - e, -1.0, -a], [b, a, -be]]
            c[k] = np.array([sg * (b - a), a * (rho - e) - b, a * b - be * e]) - F[k] @ xb[k]
        return (F, c, np.eye(3), q * np.eye(3), np.repeat(np.eye(3)[None], T, 0),
                np.zeros((T, 3)), rr * np.eye(3))
    raise ValueError(wl.model)


def joint_gaussian(wl, s, xbar=None):
    """Mean and covariance of (x_0..x_T) and of (y_1..y_T) under the discrete model."""
    F, c, L, W, H, r, R = step_terms(wl, s, xbar)
    st = wl.seg_steps(s)
    dt = wl.dt[st]
    T = len(dt)
    nx, ny = wl.nx, wl.ny
    n = (T + 1) * nx
    Q = L @ W @ L.T
    # x_k = Phi_k (x_{k-1} + dt c + w_k):  x = mu + M xi
    Phis = [np.linalg.inv(np.eye(nx) - dt[k] * F[k]) for k in range(T)]
    mu = np.zeros(n)
    mu[:nx] = wl.m0[s]
    for k in range(T):
        mu[(k + 1) * nx:(k + 2) * nx] = Phis[k] @ (mu[k * nx:(k + 1) * nx] + dt[k] * c[k])
    M = np.zeros((n, n))
    M[:nx, :nx] = np.eye(nx)
    for k in range(T):
        rows = slice((k + 1) * nx, (k + 2) * nx)
        M[rows] = Phis[k] @ M[k * nx:(k + 1) * nx]
        M[rows, (k + 1) * nx:(k + 2) * nx] += Phis[k]
    Cxi = np.zeros((n, n))
    Cxi[:nx, :nx] = wl.P0[s]
    for k in range(T):
        Cxi[(k + 1) * nx:(k + 2) * nx, (k + 1) * nx:(k + 2) * nx] = dt[k] * Q
    Sx = M @ Cxi @ M.T
    Hb = np.zeros((T * ny, n))
    Rb = np.zeros((T * ny, T * ny))
    rb = np.zeros(T * ny)
    for k in range(T):
        Hb[k * ny:(k + 1) * ny, (k + 1) * nx:(k + 2) * nx] = H[k]
        Rb[k * ny:(k + 1) * ny, k * ny:(k + 1) * ny] = R / dt[k]
        rb[k * ny:(k + 1) * ny] = r[k]
    return mu, Sx, Hb, Rb, rb


def dense_posterior(wl, s, xbar=None, upto=None):
    """Posterior mean/cov of all states given y_1..y_upto (default all), and log p(y_1..y_upto)."""
    mu, Sx, Hb, Rb, rb = joint_gaussian(wl, s, xbar)
    st = wl.seg_steps(s)
    T = st.stop - st.start
    ny = wl.ny
    upto = T if upto is None else upto
    yv = wl.y[:, st].T.reshape(-1)[:upto * ny]
    Hb, Rb, rb = Hb[:upto * ny], Rb[:upto * ny, :upto * ny], rb[:upto * ny]
    my = Hb @ mu + rb
    Sy = Hb @ Sx @ Hb.T + Rb
    Sxy = Sx @ Hb.T
    Kd = np.linalg.solve(Sy, Sxy.T).T
    mean = mu + Kd @ (yv - my)
    cov = Sx - Kd @ Sxy.T
    sign, logdet = np.linalg.slogdet(Sy)
    e = yv - my
    ll = -0.5 * (len(yv) * np.log(2 * np.pi) + logdet + e @ np.linalg.solve(Sy, e))
    return mean.reshape(T + 1, wl.nx), cov, ll


def dense_least_squares(wl, s, xbar=None):
    """argmin of the discretised objective by one dense least-squares solve
    (needs W and L invertible so that every residual has a whitening factor)."""
    F, c, L, W, H, r, R = step_terms(wl, s, xbar)
    st = wl.seg_steps(s)
    dt = wl.dt[st]
    T = len(dt)
    nx, ny = wl.nx, wl.ny
    n = (T + 1) * nx
    Q = L @ W @ L.T
    blocks, rhs = [], []
    Wp = np.linalg.cholesky(np.linalg.inv(wl.P0[s])).T
    A0 = np.zeros((nx, n)); A0[:, :nx] = Wp
    blocks.append(A0); rhs.append(Wp @ wl.m0[s])
    for k in range(T):
        h = dt[k]
        Wq = np.linalg.cholesky(np.linalg.inv(h * Q)).T
        Ak = np.zeros((nx, n))
        Ak[:, (k + 1) * nx:(k + 2) * nx] = Wq @ (np.eye(nx) - h * F[k])
        Ak[:, k * nx:(k + 1) * nx] = -Wq
        blocks.append(Ak); rhs.append(Wq @ (h * c[k]))
        Wr = np.linalg.cholesky(np.linalg.inv(R / h)).T
        Ay = np.zeros((ny, n))
        Ay[:, (k + 1) * nx:(k + 2) * nx] = Wr @ H[k]
        blocks.append(Ay); rhs.append(Wr @ (wl.y[:, st.start + k] - r[k]))
    A = np.vstack(blocks)
    b = np.concatenate(rhs)
    x, *_ = np.linalg.lstsq(A, b, rcond=None)
    res = A @ x - b
    return x.reshape(T + 1, nx), 0.5 * res @ res
