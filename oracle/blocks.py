"""Sub-stepped blocks (test infrastructure only; the product path never
imports this).

The paper's experiments (Sec. 5.1) divide the time axis into T blocks and
build each block's element by integrating the element ODE (Sec. 4.2,
eq. backwardLQT) with n explicit-Euler substeps.  Here:

  * `euler_block`  the partial elements of one block after each of its n
    substeps: the ODE written in original time, from the boundary value
    (I, 0, 0, 0, 0), substep j using the measurement at its end, with the A
    equation read as A' = -A (Q J + F) (sign_qj = -1 gives the printed
    -A Q J^T instead, for the pin that decides between them);
  * `smooth`  the filter and the MAP trajectory of a problem whose steps are
    such blocks: each element read as its conditional value function
    V(x_k, x_{k-1}) = 1/2 x_k^T J x_k - x_k^T eta + 1/2 |x_{k-1} - A x_k - b|^2_{C^-1},
    i.e. a backward transition x_{k-1} = A x_k + b + N(0, C) and an
    information term (J, eta) on x_k, and conditioned on in covariance form
    (plain Gaussian algebra with (P + C)^-1; no combination rule);
  * the dense output inside every block: the filter at each interior substep
    (the block's start carried through the partial element) and the MAP
    state there by the paper's first recovery method (Sec. 3.5, Sec. 4.3):
    the closed-loop ODE of the optimal trajectory, in original time
    dx*/dt = (F + Q S) x* - Q v + c, by explicit Euler backwards from the
    block's end, each substep with the filter at its later end.

Model terms come from `models.terms_numpy`, held over each block (evaluated
at the block's last state).
"""
from __future__ import annotations

import numpy as np

from . import models


def euler_block(F, c, Q, H, Rinv, r, ys, h, sign_qj=+1.0):
    """Partial elements [(A, b, C, eta, J) after substeps 1..n] of a block of
    len(ys) substeps of length h (ys [n, ny], the measurement at each
    substep's end)."""
    n = F.shape[0]
    A, b, C, eta, J = np.eye(n), np.zeros(n), np.zeros((n, n)), np.zeros(n), np.zeros((n, n))
    out = []
    for y in ys:
        dA = -A @ (sign_qj * Q @ J + F)
        db = A @ (Q @ eta - c)
        dC = A @ Q @ A.T
        deta = -F.T @ eta - J @ Q @ eta + J @ c + H.T @ Rinv @ (y - r)
        dJ = -F.T @ J - J @ F - J @ Q @ J + H.T @ Rinv @ H
        A, b, C, eta, J = A + h * dA, b + h * db, C + h * dC, eta + h * deta, J + h * dJ
        out.append((A.copy(), b.copy(), C.copy(), eta.copy(), J.copy()))
    return out


def _through(m, P, e):
    """Filter (m, P) at an element's earlier state carried to its later state:
    information J + A^T (P + C)^-1 A and vector eta + A^T (P + C)^-1 (m - b)."""
    A, b, C, eta, J = e
    K = np.linalg.inv(P + C)
    S = A.T @ K @ A + J
    v = A.T @ K @ (m - b) + eta
    Pn = np.linalg.inv(S)
    Pn = 0.5 * (Pn + Pn.T)
    return Pn @ v, Pn, S, v


def smooth(wl, xbar=None):
    """Filter, MAP trajectory and dense output of every segment of a workload
    whose steps are blocks of wl.n_sub substeps (y: [ny * n_sub, n_steps],
    component j * ny + c = measurement c at the end of substep j + 1).
    xbar [nx, n_states]: linearisation states (nonlinear models).
    Returns dict(m, P, S, v, xs, Ps) per state and, per state (the block ending
    there), dense_S [n-1, nx, nx], dense_v [n-1, nx], dense_m, dense_xs
    [n-1, nx] at the interior substeps."""
    nx, ny, n = wl.nx, wl.ny, wl.n_sub
    NS = wl.n_states
    if xbar is None:
        xbar = np.zeros((nx, NS))
    m_all = np.zeros((NS, nx)); P_all = np.zeros((NS, nx, nx))
    S_all = np.zeros((NS, nx, nx)); v_all = np.zeros((NS, nx))
    xs = np.zeros((NS, nx)); Ps = np.zeros((NS, nx, nx))
    dS = np.zeros((NS, n - 1, nx, nx)); dv = np.zeros((NS, n - 1, nx))
    dm = np.zeros((NS, n - 1, nx)); dx = np.zeros((NS, n - 1, nx))
    for s in range(wl.n_seg):
        st = wl.seg_steps(s)
        x0 = st.start + s
        T = st.stop - st.start
        xb = xbar[:, x0 + 1: x0 + T + 1].T
        F, c, L, W, H, r, R = models.terms_numpy(wl.model, wl.theta[s], xb, nx)
        Q = L @ W @ L.T
        Rinv = np.linalg.inv(R)
        m, P = wl.m0[s].copy(), wl.P0[s].copy()
        m_all[x0], P_all[x0] = m, P
        S_all[x0] = np.linalg.inv(P)
        v_all[x0] = S_all[x0] @ m
        elems, parts = [], []
        for k in range(T):
            Hk = H[k] if H.ndim == 3 else H
            rk = r[k] if r.ndim == 2 else r
            Fk = F[k] if F.ndim == 3 else F
            ck = c[k] if c.ndim == 2 else c
            h = wl.dt[st.start + k] / n
            ys = wl.y[:, st.start + k].reshape(n, ny)
            pe = euler_block(Fk, ck, Q, Hk, Rinv, rk, ys, h)
            parts.append((pe, Fk, ck, h))
            elems.append(pe[-1])
            m, P, S, v = _through(m, P, pe[-1])
            i = x0 + k + 1
            m_all[i], P_all[i], S_all[i], v_all[i] = m, P, S, v
        # backward: Gaussian conditioning on the backward transition of each block
        i = x0 + T
        xs[i], Ps[i] = m_all[i], P_all[i]
        for k in range(T, 0, -1):
            A, b, C, _, _ = elems[k - 1]
            i = x0 + k
            mp, Pp = m_all[i - 1], P_all[i - 1]
            G = Pp @ np.linalg.inv(Pp + C)
            xs[i - 1] = mp + G @ (A @ xs[i] + b - mp)
            Pk = Pp - G @ Pp + G @ A @ Ps[i] @ A.T @ G.T
            Ps[i - 1] = 0.5 * (Pk + Pk.T)
        # dense output inside every block
        for k in range(1, T + 1):
            i = x0 + k
            pe, Fk, ck, h = parts[k - 1]
            for j in range(1, n):
                mj, Pj, Sj, vj = _through(m_all[i - 1], P_all[i - 1], pe[j - 1])
                dS[i, j - 1], dv[i, j - 1], dm[i, j - 1] = Sj, vj, mj
            x = xs[i].copy()
            S, v = S_all[i], v_all[i]
            for j in range(n - 1, 0, -1):
                x = x - h * ((Fk + Q @ S) @ x - Q @ v + ck)
                dx[i, j - 1] = x
                S, v = dS[i, j - 1], dv[i, j - 1]
    return dict(m=m_all, P=P_all, S=S_all, v=v_all, xs=xs, Ps=Ps, dense_S=dS, dense_v=dv,
                dense_m=dm, dense_xs=dx)


def iterate(wl, n_iter=None):
    """Iterated linearisation (Sec. 4.4) over blocks from xbar^(0) = m0 at
    every state; returns the last solve's outputs with 'xbar' its
    linearisation point."""
    n_iter = wl.n_iter if n_iter is None else n_iter
    xbar = np.empty((wl.nx, wl.n_states))
    for s in range(wl.n_seg):
        xbar[:, wl.seg_states(s)] = wl.m0[s][:, None]
    out = None
    for _ in range(n_iter):
        out = smooth(wl, xbar)
        out["xbar"] = xbar
        xbar = out["xs"].T.copy()
    return out
