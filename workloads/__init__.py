"""Seeded synthetic inputs shared by the oracle-side tests and the GPU side.

This module only draws data.  It holds none of the estimation method's
arithmetic: no discretised elements, no filtering, no smoothing.  It simulates
a ground-truth path of each SDE (Euler--Maruyama on a fine grid, or an exact
linear recursion for the constant-velocity model) and draws noisy
measurements with per-sample covariance R/dt, because R is a spectral
density in the paper's problem statement (Sec. 2.1, eq. statespace).

Workloads follow the paper's experiment shapes (Sec. 5.1 Wiener velocity,
Sec. 5.2 iterated linearisation) plus the batched and nonlinear cases used
for measurement:

  cfg1  Wiener velocity, nx=2 ny=1, q=1, r=0.1, T=1024 on [0,10], m0=0, P0=I
  cfg2  2-D constant velocity, nx=4 ny=2, q=0.5, r=0.05, T=2^20, dt=1e-3,
        m0=(5,5,0,0), P0=1e-2 I
  cfg3  Van der Pol mu=1.5, q=0.1, h=x1, r=0.05, T=2^18, dt=1e-3, 10 iterations
  cfg4  4096 constant-velocity trajectories, lengths floor(2^U(8,14)),
        q~U[0.1,1], r~U[0.01,0.2], dt=1e-3
  cfg5  256 Lorenz-63 trajectories (10, 28, 8/3), q=0.5, r=0.5, T=2^14,
        full-state measurements, 5 iterations

Parameter vectors (theta) per model:
  CV        (gamma, q, r)   drift [[0,I],[0,-gamma I]], L=[0;I], W=qI, H=[I 0], R=rI
  VDP       (mu, q, r)      f=(x2, mu(1-x1^2)x2 - x1), L=I, W=qI, h=x1, R=r
  LORENZ63  (sigma, rho, beta, q, r)  L=I, W=qI, h=x, R=rI
"""
from __future__ import annotations

import dataclasses
import numpy as np
from scipy.signal import lfilter

MODEL_IDS = {"linear": 0, "cv": 1, "vdp": 2, "lorenz63": 3, "ct": 4}
N_THETA = {"cv": 3, "vdp": 3, "lorenz63": 5, "ct": 4}


@dataclasses.dataclass
class Workload:
    name: str
    model: str                 # "cv" | "vdp" | "lorenz63" | "ct" | "linear"
    nx: int
    ny: int
    nw: int
    seg_off: np.ndarray        # int64 [n_seg+1] step offsets
    dt: np.ndarray             # float64 [n_steps] (uniform grids are still stored per step)
    y: np.ndarray              # float64 [ny, n_steps] measurement of the step's right-end state
    theta: np.ndarray          # float64 [n_seg, n_theta]
    m0: np.ndarray             # float64 [n_seg, nx]
    P0: np.ndarray             # float64 [n_seg, nx, nx]
    x_true: np.ndarray         # float64 [nx, n_states] simulated path (states, per segment T+1)
    n_iter: int = 1            # Gauss--Newton iterations (1 for linear models)
    dtype: str = "f64"
    lin: dict | None = None    # model "linear": F [nx,nx] or [n_steps,nx,nx], c, L, W, H, r, R
    n_sub: int = 1             # substeps per step (blocks): y is then [ny * n_sub, n_steps]

    @property
    def n_seg(self) -> int:
        return int(self.seg_off.shape[0] - 1)

    @property
    def n_steps(self) -> int:
        return int(self.seg_off[-1])

    @property
    def n_states(self) -> int:
        return self.n_steps + self.n_seg

    def seg_steps(self, s: int) -> slice:
        return slice(int(self.seg_off[s]), int(self.seg_off[s + 1]))

    def seg_states(self, s: int) -> slice:
        return slice(int(self.seg_off[s]) + s, int(self.seg_off[s + 1]) + s + 1)

    def rounded(self, dtype: str) -> "Workload":
        """Copy whose real inputs are rounded to `dtype` (stored back in float64),
        so that an FP32 run and the FP64 oracle see identical inputs."""
        if dtype == "f64":
            return dataclasses.replace(self, dtype="f64")
        r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        lin = None if self.lin is None else {k: r(v) for k, v in self.lin.items()}
        return dataclasses.replace(self, dt=r(self.dt), y=r(self.y), theta=r(self.theta),
                                   m0=r(self.m0), P0=r(self.P0), dtype=dtype, lin=lin)


def blocks(wl: Workload, n_sub: int) -> Workload:
    """The same data regrouped into blocks of n_sub consecutive steps (each
    segment's length must be a multiple of n_sub): a block's step length is
    the sum of its substeps' (uniform within a block), its measurements are
    those of its substeps in order (y [ny * n_sub, n_blocks], component
    j * ny + c = measurement c at the end of substep j + 1), and x_true keeps
    the block boundaries."""
    lens = np.diff(wl.seg_off)
    if np.any(lens % n_sub):
        raise ValueError("segment lengths must be multiples of n_sub")
    nb = lens // n_sub
    seg_off = np.zeros_like(wl.seg_off)
    seg_off[1:] = np.cumsum(nb)
    ny = wl.ny
    y = wl.y.T.reshape(-1, n_sub * ny).T.copy()
    dt = wl.dt.reshape(-1, n_sub).sum(1)
    keep = np.concatenate([wl.seg_off[s] + s + n_sub * np.arange(nb[s] + 1)
                           for s in range(wl.n_seg)])
    return dataclasses.replace(wl, name=wl.name + "_blocks%d" % n_sub, seg_off=seg_off, dt=dt,
                               y=y, x_true=wl.x_true[:, keep], n_sub=n_sub)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _cv_path(rng, T, d, dt, gamma, q, x0):
    """Exact-in-distribution simulation of the damped constant-velocity SDE
    dv = -gamma v dt + sqrt(q) dB, dp = v dt on a uniform grid (velocity as an
    AR(1) recursion, position as its running integral)."""
    a = np.exp(-gamma * dt)
    var = q * dt if gamma == 0.0 else q * (1.0 - a * a) / (2.0 * gamma)
    x = np.empty((2 * d, T + 1))
    x[:, 0] = x0
    for i in range(d):
        w = rng.standard_normal(T) * np.sqrt(var)
        v = lfilter([1.0], [1.0, -a], w, zi=np.array([a * x0[d + i]]))[0]
        x[d + i, 1:] = v
        x[i, 1:] = x0[i] + np.cumsum(v) * dt
    return x


def _em_path(rng, T, dt, drift, nx, q, x0, substeps):
    """Euler--Maruyama with `substeps` substeps per grid step, diffusion sqrt(q) I."""
    h = dt / substeps
    x = np.empty((nx, T + 1))
    cur = np.array(x0, dtype=np.float64)
    x[:, 0] = cur
    noise = rng.standard_normal((T, substeps, nx)) * np.sqrt(q * h)
    for k in range(T):
        for j in range(substeps):
            cur = cur + h * drift(cur) + noise[k, j]
        x[:, k + 1] = cur
    return x


def _em_batch(rng, n, T, dt, drift, nx, q, x0, substeps):
    """Vectorised over n trajectories: x [n, nx, T+1]."""
    h = dt / substeps
    x = np.empty((n, nx, T + 1))
    cur = np.array(x0, dtype=np.float64).reshape(n, nx)
    x[:, :, 0] = cur
    for k in range(T):
        for j in range(substeps):
            cur = cur + h * drift(cur) + rng.standard_normal((n, nx)) * np.sqrt(q * h)
        x[:, :, k + 1] = cur
    return x


def _measure(rng, hx, dt, r):
    """y = h(x) + noise with per-sample covariance r/dt (R is a spectral density)."""
    return hx + rng.standard_normal(hx.shape) * np.sqrt(r / dt)


def cv(T=1024, d=1, dt=None, t_end=None, gamma=0.0, q=1.0, r=0.1, m0=None, P0=None,
       seed=1, name="cv") -> Workload:
    if dt is None:
        dt = t_end / T
    nx = 2 * d
    rng = _rng(seed)
    m0 = np.zeros(nx) if m0 is None else np.asarray(m0, dtype=np.float64)
    P0 = np.eye(nx) if P0 is None else np.asarray(P0, dtype=np.float64)
    x0 = rng.multivariate_normal(m0, P0)
    x = _cv_path(rng, T, d, dt, gamma, q, x0)
    y = _measure(rng, x[:d, 1:], dt, r)
    return Workload(name=name, model="cv", nx=nx, ny=d, nw=d,
                    seg_off=np.array([0, T], dtype=np.int64), dt=np.full(T, dt),
                    y=y, theta=np.array([[gamma, q, r]]), m0=m0[None], P0=P0[None], x_true=x)


def cv_batched(n_seg=4096, lmin=8.0, lmax=14.0, d=2, dt=1e-3, gamma=0.0,
               qrange=(0.1, 1.0), rrange=(0.01, 0.2), m0=(5, 5, 0, 0), P0=1e-2,
               seed=4, name="cv_batched", lens=None) -> Workload:
    """Segment lengths floor(2^U(lmin, lmax)) steps, or the given `lens`."""
    rng = _rng(seed)
    nx = 2 * d
    if lens is None:
        lens = np.floor(2.0 ** rng.uniform(lmin, lmax, n_seg)).astype(np.int64)
        lens = np.maximum(lens, 1)
    else:
        lens = np.asarray(lens, dtype=np.int64)
        n_seg = len(lens)
    seg_off = np.zeros(n_seg + 1, dtype=np.int64)
    seg_off[1:] = np.cumsum(lens)
    qs = rng.uniform(*qrange, n_seg)
    rs = rng.uniform(*rrange, n_seg)
    m0v = np.asarray(m0, dtype=np.float64)[:nx]
    P0m = np.eye(nx) * P0
    y = np.empty((d, seg_off[-1]))
    xs = np.empty((nx, seg_off[-1] + n_seg))
    for s in range(n_seg):
        x0 = rng.multivariate_normal(m0v, P0m)
        x = _cv_path(rng, int(lens[s]), d, dt, gamma, qs[s], x0)
        xs[:, seg_off[s] + s: seg_off[s + 1] + s + 1] = x
        y[:, seg_off[s]:seg_off[s + 1]] = _measure(rng, x[:d, 1:], dt, rs[s])
    theta = np.stack([np.full(n_seg, gamma), qs, rs], axis=1)
    return Workload(name=name, model="cv", nx=nx, ny=d, nw=d, seg_off=seg_off,
                    dt=np.full(int(seg_off[-1]), dt), y=y, theta=theta,
                    m0=np.tile(m0v, (n_seg, 1)), P0=np.tile(P0m, (n_seg, 1, 1)), x_true=xs)


def vdp(T=2 ** 18, dt=1e-3, mu=1.5, q=0.1, r=0.05, m0=(2.0, 0.0), P0=0.1, n_iter=10,
        substeps=4, seed=3, name="vdp") -> Workload:
    rng = _rng(seed)
    m0 = np.asarray(m0, dtype=np.float64)
    P0m = np.eye(2) * P0
    drift = lambda x: np.array([x[1], mu * (1.0 - x[0] ** 2) * x[1] - x[0]])
    x0 = rng.multivariate_normal(m0, P0m)
    x = _em_path(rng, T, dt, drift, 2, q, x0, substeps)
    y = _measure(rng, x[:1, 1:], dt, r)
    return Workload(name=name, model="vdp", nx=2, ny=1, nw=2,
                    seg_off=np.array([0, T], dtype=np.int64), dt=np.full(T, dt), y=y,
                    theta=np.array([[mu, q, r]]), m0=m0[None], P0=P0m[None], x_true=x,
                    n_iter=n_iter)


def lorenz63(n_seg=256, T=2 ** 14, dt=1e-3, sigma=10.0, rho=28.0, beta=8.0 / 3.0, q=0.5,
             r=0.5, m0=(1.0, 1.0, 1.0), P0=1.0, n_iter=5, substeps=4, seed=5,
             name="lorenz63") -> Workload:
    rng = _rng(seed)
    m0 = np.asarray(m0, dtype=np.float64)
    P0m = np.eye(3) * P0

    def drift(x):
        return np.stack([sigma * (x[:, 1] - x[:, 0]),
                         x[:, 0] * (rho - x[:, 2]) - x[:, 1],
                         x[:, 0] * x[:, 1] - beta * x[:, 2]], axis=1)

    x0 = rng.multivariate_normal(m0, P0m, size=n_seg)
    X = _em_batch(rng, n_seg, T, dt, drift, 3, q, x0, substeps)
    seg_off = np.arange(n_seg + 1, dtype=np.int64) * T
    y = np.empty((3, n_seg * T))
    xs = np.empty((3, n_seg * (T + 1)))
    for s in range(n_seg):
        xs[:, s * (T + 1):(s + 1) * (T + 1)] = X[s]
        y[:, s * T:(s + 1) * T] = _measure(rng, X[s][:, 1:], dt, r)
    theta = np.tile(np.array([sigma, rho, beta, q, r]), (n_seg, 1))
    return Workload(name=name, model="lorenz63", nx=3, ny=3, nw=3, seg_off=seg_off,
                    dt=np.full(n_seg * T, dt), y=y, theta=theta,
                    m0=np.tile(m0, (n_seg, 1)), P0=np.tile(P0m, (n_seg, 1, 1)), x_true=xs,
                    n_iter=n_iter)


def ct(n_seg=64, T=2 ** 14, dt=1e-3, sv=5e-4, sw=0.02, r=(5e-3, 1e-3),
       m0=(5.0, 5.0, 0.0, 0.3, 0.0), P0=(0.01, 0.01, 0.01, 0.01, 0.04), n_iter=5, seed=6,
       name="ct") -> Workload:
    """Coordinated-turn tracks with the parameters of the paper's nonlinear
    experiment (Sec. 5.2): x = (xi, zeta, dxi, dzeta, omega), turn rate a random
    walk with spectral density sw^2, velocity rotated at the turn rate plus
    white acceleration with density sv^2, range and bearing measured with
    spectral densities r (per-sample covariance r/dt), bearings reported in
    [-pi, pi).  The velocity is simulated with an exponential integrator of the
    rotation: with z = dxi + i dzeta and phase Phi_k = dt sum_{j<k} omega_j,
    z_k = exp(i Phi_k) (z_0 + sum_{j<k} exp(-i Phi_{j+1}) sv dB_j); position is
    the running sum of dt z."""
    rng = _rng(seed)
    m0 = np.asarray(m0, dtype=np.float64)
    P0m = np.diag(np.asarray(P0, dtype=np.float64))
    seg_off = np.arange(n_seg + 1, dtype=np.int64) * T
    y = np.empty((2, n_seg * T))
    xs = np.empty((5, n_seg * (T + 1)))
    for s in range(n_seg):
        x0 = rng.multivariate_normal(m0, P0m)
        om = x0[4] + np.concatenate([[0.0], np.cumsum(rng.standard_normal(T) * sw * np.sqrt(dt))])
        phase = np.concatenate([[0.0], np.cumsum(om[:-1] * dt)])           # Phi_0..Phi_T
        dB = (rng.standard_normal(T) + 1j * rng.standard_normal(T)) * sv * np.sqrt(dt)
        acc = np.concatenate([[0.0], np.cumsum(np.exp(-1j * phase[1:]) * dB)])
        z = np.exp(1j * phase) * (x0[2] + 1j * x0[3] + acc)
        p = (x0[0] + 1j * x0[1]) + np.concatenate([[0.0], np.cumsum(z[1:] * dt)])
        X = np.stack([p.real, p.imag, z.real, z.imag, om])
        xs[:, s * (T + 1):(s + 1) * (T + 1)] = X
        rng_ = np.hypot(X[0, 1:], X[1, 1:])
        brg = np.arctan2(X[1, 1:], X[0, 1:])
        yy = _measure(rng, np.stack([rng_, brg]), dt, np.asarray(r, dtype=np.float64)[:, None])
        yy[1] = yy[1] - 2.0 * np.pi * np.floor(yy[1] / (2.0 * np.pi) + 0.5)
        y[:, s * T:(s + 1) * T] = yy
    theta = np.tile(np.array([sv, sw, r[0], r[1]]), (n_seg, 1))
    return Workload(name=name, model="ct", nx=5, ny=2, nw=3, seg_off=seg_off,
                    dt=np.full(n_seg * T, dt), y=y, theta=theta,
                    m0=np.tile(m0, (n_seg, 1)), P0=np.tile(P0m, (n_seg, 1, 1)), x_true=xs,
                    n_iter=n_iter)


def linear_random(T=64, nx=3, ny=2, nw=2, dt=0.05, time_varying=True, n_seg=1,
                  seed=11, name="linear_random", stable=False) -> Workload:
    """A general time-varying linear-affine model (Sec. 2.4, eq. linear-statespace)
    with c != 0 and r != 0, dense F, L, H: F_k = F0 + 0.3 sin(0.1 k) F1,
    c_k = c0 cos(0.05 k), H_k = H0 + 0.2 cos(0.07 k) H1, r_k = r0 (1 + 0.5 sin(0.03 k)).
    L, W, R are shared by all steps.  All segments have length T and share
    the model; their data differ.  `stable` shifts F0 so that its eigenvalues
    have real part at most -0.5 (a random F0 grows without bound otherwise,
    more often the larger nx, and long segments then reach magnitudes where
    rounding of the state, not the method, sets the error of the
    log-likelihood)."""
    rng = _rng(seed)
    F0 = rng.standard_normal((nx, nx)) * 0.6 - 0.5 * np.eye(nx)
    if stable:
        F0 -= max(np.linalg.eigvals(F0).real.max() + 0.5, 0.0) * np.eye(nx)
    F1 = rng.standard_normal((nx, nx)) * 0.4
    c0 = rng.standard_normal(nx)
    H0 = rng.standard_normal((ny, nx))
    H1 = rng.standard_normal((ny, nx))
    r0 = rng.standard_normal(ny)
    L = rng.standard_normal((nx, nw))
    Wh = rng.standard_normal((nw, nw)) * 0.3
    W = Wh @ Wh.T + 0.5 * np.eye(nw)
    Rh = rng.standard_normal((ny, ny)) * 0.1
    R = Rh @ Rh.T + 0.05 * np.eye(ny)
    N = T * n_seg
    kk = np.tile(np.arange(T), n_seg).astype(np.float64)
    if time_varying:
        F = F0[None] + 0.3 * np.sin(0.1 * kk)[:, None, None] * F1[None]
        c = c0[None] * np.cos(0.05 * kk)[:, None]
        H = H0[None] + 0.2 * np.cos(0.07 * kk)[:, None, None] * H1[None]
        r = r0[None] * (1.0 + 0.5 * np.sin(0.03 * kk))[:, None]
    else:
        F = np.broadcast_to(F0, (N, nx, nx)).copy()
        c = np.broadcast_to(c0, (N, nx)).copy()
        H = np.broadcast_to(H0, (N, ny, nx)).copy()
        r = np.broadcast_to(r0, (N, ny)).copy()
    m0 = rng.standard_normal(nx)
    Ph = rng.standard_normal((nx, nx)) * 0.3
    P0 = Ph @ Ph.T + 0.2 * np.eye(nx)
    Wc = np.linalg.cholesky(W)
    seg_off = np.arange(n_seg + 1, dtype=np.int64) * T
    y = np.empty((ny, N))
    xs = np.empty((nx, N + n_seg))
    sub = 8
    for s in range(n_seg):
        x = rng.multivariate_normal(m0, P0)
        xs[:, s * (T + 1)] = x
        for j in range(T):
            k = s * T + j
            for _ in range(sub):
                h = dt / sub
                x = x + h * (F[k] @ x + c[k]) + np.sqrt(h) * (L @ (Wc @ rng.standard_normal(nw)))
            xs[:, s * (T + 1) + j + 1] = x
            y[:, k] = H[k] @ x + r[k] + rng.multivariate_normal(np.zeros(ny), R / dt)
    lin = dict(F=F, c=c, L=L, W=W, H=H, r=r, R=R)
    return Workload(name=name, model="linear", nx=nx, ny=ny, nw=nw, seg_off=seg_off,
                    dt=np.full(N, dt), y=y, theta=np.zeros((n_seg, 0)),
                    m0=np.tile(m0, (n_seg, 1)), P0=np.tile(P0, (n_seg, 1, 1)), x_true=xs, lin=lin)


def config(n: int, scale: float = 1.0) -> Workload:
    """The five named workloads.  `scale` < 1 shrinks the time axis (and the
    number of trajectories of cfg4/cfg5) for quick parity cases."""
    if n == 1:
        return cv(T=1024, d=1, t_end=10.0, q=1.0, r=0.1, seed=1, name="cfg1_wiener_velocity")
    if n == 2:
        T = max(16, int(2 ** 20 * scale))
        return cv(T=T, d=2, dt=1e-3, q=0.5, r=0.05, m0=[5, 5, 0, 0], P0=1e-2 * np.eye(4),
                  seed=2, name="cfg2_cv2d")
    if n == 3:
        T = max(16, int(2 ** 18 * scale))
        return vdp(T=T, seed=3, name="cfg3_vdp")
    if n == 4:
        ns = max(2, int(4096 * scale))
        return cv_batched(n_seg=ns, seed=4, name="cfg4_cv_batched")
    if n == 5:
        ns = max(2, int(256 * scale))
        T = max(16, int(2 ** 14 * min(1.0, scale * 4)))
        return lorenz63(n_seg=ns, T=T, seed=5, name="cfg5_lorenz63")
    raise ValueError(n)
