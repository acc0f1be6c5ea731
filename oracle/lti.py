"""Exact discretisation of a time-invariant linear-affine model (test
infrastructure only; never imported by the product path).

For dx/dt = F x + c + L w (w white, spectral density W) the transition over
dt is x_k = Phi x_{k-1} + u + w_k with Phi = e^{F dt},
u = int_0^dt e^{F s} ds c and w_k ~ N(0, Qd), Qd = int_0^dt e^{F s} Q e^{F^T s} ds,
Q = L W L^T (Van Loan: the exponential of [[-F, Q], [0, F^T]] dt has
e^{F^T dt} in its lower-right block and e^{-F dt} Qd in its upper-right one).  Written backwards, x_{k-1} = A x_k + b + noise
with A = e^{-F dt}, b = -A u and covariance C = A Qd A^T: these are the exact
dynamics parts of the one-step element (Sec. 4.2 integrates eq. backwardLQT
with the measurement term exactly over the step when H = 0).

`implicit_equivalent` re-expresses (A, b, C) in the terms of the oracle's
implicit-Euler step (kfs.c): F~ = (I - A) / dt, c~ = -b / dt, and any L~ with
L~ L~^T = C / dt (W~ = I), so that the same sequential filter and smoother
solve the exactly discretised problem.  Here L~ comes from a symmetric
eigendecomposition.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def van_loan(F, c, L, W, dt):
    """Phi, u, Qd of the exact transition over dt (scipy's expm)."""
    n = F.shape[0]
    Q = L @ W @ L.T
    M = np.zeros((2 * n, 2 * n))
    M[:n, :n] = -F
    M[:n, n:] = Q
    M[n:, n:] = F.T
    E = scipy.linalg.expm(M * dt)
    Phi = E[n:, n:].T
    Qd = Phi @ E[:n, n:]
    Qd = 0.5 * (Qd + Qd.T)
    Mu = np.zeros((n + 1, n + 1))
    Mu[:n, :n] = F
    Mu[:n, n] = c
    u = scipy.linalg.expm(Mu * dt)[:n, n]
    return Phi, u, Qd


def implicit_equivalent(F, c, L, W, dt):
    """(F~, c~, L~, W~ = I) whose implicit-Euler step over dt is the exact transition."""
    n = F.shape[0]
    Phi, u, Qd = van_loan(F, c, L, W, dt)
    A = np.linalg.inv(Phi)
    b = -A @ u
    C = A @ Qd @ A.T
    C = 0.5 * (C + C.T)
    lam, U = np.linalg.eigh(C / dt)
    Lt = U * np.sqrt(np.maximum(lam, 0.0))
    return (np.eye(n) - A) / dt, -b / dt, Lt, np.eye(n)
