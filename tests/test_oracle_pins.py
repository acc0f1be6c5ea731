"""Pins of the CPU oracle against things that do not come from the oracle.

Each test names what fixes the expected value: dense Gaussian conditioning
of the discrete model, dense least squares of the discretised
Onsager--Machlup objective, the discrete algebraic Riccati equation, the
closed-form continuous-time Riccati solution of the Wiener velocity model,
central finite differences of a dense likelihood, and nonlinear least squares.
Every linear case has c != 0 and r != 0 somewhere (an S_k / S_{k-1} slip in
an information-vector update only shows when the element offset b is
nonzero).
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import torch

import workloads
from oracle import blocks as oracle_blocks
from oracle import cref, ref
from tests import _dense

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _cases():
    return [
        workloads.linear_random(T=24, nx=3, ny=2, nw=3, seed=21),          # dense Q, c, r != 0
        workloads.linear_random(T=20, nx=4, ny=2, nw=2, seed=22),          # singular Q
        workloads.cv(T=18, d=2, dt=0.05, gamma=0.4, q=0.5, r=0.05, m0=[5, 5, 0, 0],
                     P0=1e-2 * np.eye(4), seed=23),                         # CV, singular Q
        workloads.linear_random(T=16, nx=2, ny=1, nw=2, seed=24, time_varying=False),
    ]


@pytest.mark.parametrize("case", range(4))
def test_smoother_equals_dense_conditioning(case):
    wl = _cases()[case]
    o = cref.smooth(wl)
    mean, cov, ll = _dense.dense_posterior(wl, 0)
    T = wl.n_steps
    nx = wl.nx
    assert np.abs(o["xs"] - mean).max() <= 1e-11 * max(1.0, np.abs(mean).max())
    dcov = np.stack([cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(T + 1)])
    assert np.abs(o["Ps"] - dcov).max() <= 1e-11 * max(1.0, np.abs(dcov).max())
    assert abs(o["loglik"][0] - ll) <= 1e-10 * max(1.0, abs(ll))


@pytest.mark.parametrize("case", range(4))
def test_filter_equals_dense_conditioning(case):
    wl = _cases()[case]
    o = cref.smooth(wl)
    nx = wl.nx
    for k in (1, wl.n_steps // 2, wl.n_steps):
        mean, cov, _ = _dense.dense_posterior(wl, 0, upto=k)
        assert np.abs(o["m"][k] - mean[k]).max() <= 1e-11 * max(1.0, np.abs(mean).max())
        ck = cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx]
        assert np.abs(o["P"][k] - ck).max() <= 1e-11 * max(1.0, np.abs(ck).max())


@pytest.mark.parametrize("case", [0, 3])
def test_map_estimate_equals_dense_least_squares(case):
    """With invertible Q the smoother mean is the minimiser of the discretised
    objective and M* its minimum value."""
    wl = _cases()[case]
    o = cref.smooth(wl)
    x, val = _dense.dense_least_squares(wl, 0)
    assert np.abs(o["xs"] - x).max() <= 1e-10 * max(1.0, np.abs(x).max())
    assert abs(o["mstar"][0] - val) <= 1e-10 * max(1.0, abs(val))


def test_mstar_singular_q_equals_conditioned_limit():
    """For singular Q, M* is the limit of the invertible-Q minimum value as the
    missing noise directions vanish: check continuity against a tiny added W
    direction (dense least squares on a full-rank L)."""
    wl = workloads.cv(T=16, d=1, dt=0.1, gamma=0.3, q=0.7, r=0.2, seed=31)
    o = cref.smooth(wl)
    vals = []
    for eps in (1e-6, 1e-7):
        wl2 = workloads.linear_random(T=16, nx=2, ny=1, nw=2, seed=1)
        F, c, L, W, H, r, R = _dense.step_terms(wl, 0)
        T = wl.n_steps
        lin = dict(F=F, c=c, L=np.eye(2), W=np.diag([eps, wl.theta[0, 1]]), H=H, r=r, R=R)
        wl2.lin = lin
        wl2.y, wl2.dt, wl2.m0, wl2.P0 = wl.y, wl.dt, wl.m0, wl.P0
        wl2.seg_off = wl.seg_off
        vals.append(_dense.dense_least_squares(wl2, 0)[1])
    assert abs(vals[1] - o["mstar"][0]) <= 1e-4 * abs(o["mstar"][0])
    assert abs(vals[1] - o["mstar"][0]) < abs(vals[0] - o["mstar"][0])


def test_torch_and_c_oracles_agree_on_batches():
    wl = workloads.cv_batched(n_seg=5, lmin=3, lmax=6, seed=41)
    o = cref.smooth(wl)
    for s in range(wl.n_seg):
        seg = ref.workload_segment(wl, s)
        T = wl.seg_off[s + 1] - wl.seg_off[s]
        r = ref.smooth_segment("cv", seg["theta"], torch.zeros(T + 1, 4, dtype=torch.float64),
                               seg["dt"], seg["y"], seg["m0"], seg["P0"], 4)
        st = wl.seg_states(s)
        np.testing.assert_allclose(o["xs"][st], r["xs"].numpy(), rtol=0, atol=1e-12)
        np.testing.assert_allclose(o["P"][st], r["P"].numpy(), rtol=0, atol=1e-12)
        assert abs(o["loglik"][s] - r["loglik"].item()) < 1e-10 * abs(o["loglik"][s])
        assert abs(o["mstar"][s] - r["mstar"].item()) < 1e-10 * abs(o["mstar"][s])


def test_filter_converges_to_dare():
    """Long-run filter covariance equals the discrete algebraic Riccati
    solution of the forward model (Phi, Phi dtQ Phi^T, H, R/dt)."""
    wl = workloads.cv(T=20000, d=2, dt=1e-3, q=0.5, r=0.05, m0=[5, 5, 0, 0],
                      P0=1e-2 * np.eye(4), seed=2)
    o = cref.smooth(wl)
    F, c, L, W, H, r, R = _dense.step_terms(wl, 0)
    dt = 1e-3
    Phi = np.linalg.inv(np.eye(4) - dt * F[0])
    Qd = Phi @ (dt * L @ W @ L.T) @ Phi.T
    Pp = scipy.linalg.solve_discrete_are(Phi.T, H[0].T, Qd, R / dt)
    Hk = H[0]
    Pf = Pp - Pp @ Hk.T @ np.linalg.solve(Hk @ Pp @ Hk.T + R / dt, Hk @ Pp)
    assert np.abs(o["P"][-1] - Pf).max() <= 1e-10 * np.abs(Pf).max()


def test_wiener_velocity_care_closed_form_first_order():
    """Kalman--Bucy steady state of the Wiener velocity model (Sec. 2.5):
    P_inf = [[sqrt2 q^1/4 r^3/4, sqrt(q r)], [sqrt(q r), sqrt2 q^3/4 r^1/4]].
    The discrete filter reaches it with an O(dt) error."""
    q, r = 1.0, 0.1
    Pinf = np.array([[np.sqrt(2) * q ** 0.25 * r ** 0.75, np.sqrt(q * r)],
                     [np.sqrt(q * r), np.sqrt(2) * q ** 0.75 * r ** 0.25]])
    # the closed form itself solves the CARE F P + P F^T + Q - P H^T R^-1 H P = 0
    Fm = np.array([[0.0, 1.0], [0.0, 0.0]])
    Qm = np.diag([0.0, q])
    Hm = np.array([[1.0, 0.0]])
    res = Fm @ Pinf + Pinf @ Fm.T + Qm - Pinf @ Hm.T @ Hm @ Pinf / r
    assert np.abs(res).max() < 1e-12
    errs = []
    for dt in (0.02, 0.01, 0.005):
        T = int(round(40.0 / dt))
        wl = workloads.cv(T=T, d=1, dt=dt, q=q, r=r, seed=1)
        o = cref.smooth(wl)
        errs.append(np.abs(o["P"][-1] - Pinf).max())
    assert errs[0] > errs[1] > errs[2]
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


def _dense_ll_theta(wl, theta):
    w = workloads.Workload(**{**wl.__dict__})
    w.theta = theta[None]
    return _dense.dense_posterior(w, 0)[2]


def _dense_mstar_theta(wl, theta):
    """M* = objective at the dense posterior mean (conditioning, not least
    squares, so singular Q is fine); the objective is evaluated with the
    driving-noise energy of the constrained step residuals."""
    w = workloads.Workload(**{**wl.__dict__})
    w.theta = theta[None]
    mean, _, _ = _dense.dense_posterior(w, 0)
    F, c, L, W, H, r, R = _dense.step_terms(w, 0)
    dt = w.dt
    d0 = mean[0] - w.m0[0]
    M = 0.5 * d0 @ np.linalg.solve(w.P0[0], d0)
    Lp = np.linalg.pinv(L)
    for k in range(1, mean.shape[0]):
        D = mean[k] - mean[k - 1] - dt[k - 1] * (F[k - 1] @ mean[k] + c[k - 1])
        u = Lp @ D
        e = w.y[:, k - 1] - H[k - 1] @ mean[k] - r[k - 1]
        M += 0.5 * u @ np.linalg.solve(dt[k - 1] * W, u) + 0.5 * dt[k - 1] * e @ np.linalg.solve(R, e)
    return M


@pytest.mark.parametrize("gamma", [0.0, 0.6])
def test_gradients_autograd_vs_dense_finite_differences(gamma):
    """Oracle gradients (autograd of the KF/RTS definitions) against central
    differences of the dense likelihood and of the dense objective value."""
    wl = workloads.cv(T=30, d=2, dt=0.05, gamma=gamma, q=0.5, r=0.05, m0=[5, 5, 0, 0],
                      P0=1e-2 * np.eye(4), seed=51)
    seg = ref.workload_segment(wl, 0)
    gl, gm, _ = ref.gradients("cv", 4, seg, torch.zeros(31, 4, dtype=torch.float64))
    th = wl.theta[0].copy()
    for i in range(3):
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd_l = (_dense_ll_theta(wl, tp) - _dense_ll_theta(wl, tm)) / (2 * h)
        fd_m = (_dense_mstar_theta(wl, tp) - _dense_mstar_theta(wl, tm)) / (2 * h)
        assert abs(gl[i].item() - fd_l) <= 1e-6 * max(1.0, abs(fd_l)), (i, gl[i].item(), fd_l)
        assert abs(gm[i].item() - fd_m) <= 1e-6 * max(1.0, abs(fd_m)), (i, gm[i].item(), fd_m)


def _dense_mean_theta(wl, theta, xbar=None):
    w = workloads.Workload(**{**wl.__dict__})
    w.theta = theta[None]
    return _dense.dense_posterior(w, 0, xbar)[0]


@pytest.mark.parametrize("model", ["cv", "vdp"])
def test_trajectory_vjp_vs_dense_finite_differences(model):
    """Oracle VJP of the MAP trajectory (autograd through the KF/RTS
    definitions) against central differences of the dense posterior mean
    (Gaussian conditioning of the whole discrete model), w . dx*/dtheta for a
    random cotangent w; Van der Pol with its linearisation point held fixed."""
    if model == "cv":
        wl = workloads.cv(T=25, d=2, dt=0.05, gamma=0.3, q=0.5, r=0.05, m0=[5, 5, 0, 0],
                          P0=1e-2 * np.eye(4), seed=52)
        xbar = np.zeros((4, 26))
    else:
        wl = workloads.vdp(T=25, dt=0.02, seed=53, n_iter=2)
        xbar = cref.iterate(wl, n_iter=1)["xs"].T.copy()
    nx = wl.nx
    rng = np.random.default_rng(54)
    wv = rng.normal(size=(wl.n_states, nx))
    seg = ref.workload_segment(wl, 0)
    g = ref.trajectory_vjp(model, nx, seg, torch.tensor(xbar.T.copy()),
                           torch.tensor(wv)).numpy()
    th = wl.theta[0].copy()
    for i in range(th.size):
        h = 1e-5 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = ((_dense_mean_theta(wl, tp, xbar) - _dense_mean_theta(wl, tm, xbar)) * wv).sum() / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_nonlinear_iteration_matches_nonlinear_least_squares():
    """Gauss--Newton (Sec. 4.4) on Van der Pol (Q invertible) converges to the
    minimiser of the nonlinear discretised objective found by a generic
    trust-region least-squares solver, and the objective decreases."""
    wl = workloads.vdp(T=60, dt=0.02, seed=61, n_iter=8)
    seg = ref.workload_segment(wl, 0)
    its, out = ref.gauss_newton("vdp", seg["theta"], seg["dt"], seg["y"], seg["m0"], seg["P0"],
                                2, 8)
    obj = [ref.map_objective_nonlinear("vdp", seg["theta"], x, seg["dt"], seg["y"], seg["m0"],
                                       seg["P0"], 2).item() for x in its]
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(obj[1:], obj[2:]))
    mu, q, rr = wl.theta[0]
    T = wl.n_steps
    dt = wl.dt[0]
    y = wl.y[0]
    P0i = np.linalg.cholesky(np.linalg.inv(wl.P0[0])).T

    def resid(z):
        x = z.reshape(T + 1, 2)
        out = [P0i @ (x[0] - wl.m0[0])]
        f = np.stack([x[1:, 1], mu * (1 - x[1:, 0] ** 2) * x[1:, 1] - x[1:, 0]], 1)
        D = (x[1:] - x[:-1] - dt * f) / np.sqrt(dt * q)
        E = (y - x[1:, 0]) * np.sqrt(dt / rr)
        return np.concatenate([out[0], D.reshape(-1), E])

    sol = scipy.optimize.least_squares(resid, its[-1].numpy().reshape(-1) + 0.01, xtol=1e-15,
                                       ftol=1e-15, gtol=1e-15)
    x_ls = sol.x.reshape(T + 1, 2)
    assert np.abs(its[-1].numpy() - x_ls).max() < 1e-7 * np.abs(x_ls).max()
    # stationarity of the nonlinear objective at the last iterate
    x = its[-1].clone().requires_grad_(True)
    M = ref.map_objective_nonlinear("vdp", seg["theta"], x, seg["dt"], seg["y"], seg["m0"],
                                    seg["P0"], 2)
    g, = torch.autograd.grad(M, x)
    assert g.abs().max().item() < 1e-6


def test_lorenz_iterates_c_and_torch_agree_and_decrease():
    wl = workloads.lorenz63(n_seg=2, T=200, seed=71, n_iter=5)
    o = cref.iterate(wl, keep_iterates=True)
    for s in range(2):
        seg = ref.workload_segment(wl, s)
        its, out = ref.gauss_newton("lorenz63", seg["theta"], seg["dt"], seg["y"], seg["m0"],
                                    seg["P0"], 3, 5)
        st = wl.seg_states(s)
        for i in range(5):
            np.testing.assert_allclose(o["iterates"][i][:, st].T, its[i].numpy(), rtol=0,
                                       atol=1e-9 * np.abs(its[i].numpy()).max())
        obj = [ref.map_objective_nonlinear("lorenz63", seg["theta"], x, seg["dt"], seg["y"],
                                           seg["m0"], seg["P0"], 3).item() for x in its]
        assert obj[-1] <= obj[1]


# ------------------------------------------------------------------ two-filter smoother
def _tf_cases():
    return _cases() + [
        workloads.cv_batched(lens=[9, 1, 14], d=2, dt=0.05, seed=25),       # segments, T = 1
        workloads.linear_random(T=12, nx=2, ny=2, nw=1, seed=26, n_seg=2),  # H square
    ]


@pytest.mark.parametrize("case", range(6))
def test_two_filter_equals_dense_conditioning(case):
    """Sec. 4.3 eq. twofilter: forward value function combined with the
    conditional value function of the later steps gives the posterior of the
    discrete model, state by state (dense conditioning of the joint Gaussian)."""
    wl = _tf_cases()[case]
    o = cref.two_filter(wl)
    nx = wl.nx
    for s in range(wl.n_seg):
        mean, cov, _ = _dense.dense_posterior(wl, s)
        st = wl.seg_states(s)
        T = st.stop - st.start - 1
        dcov = np.stack([cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(T + 1)])
        assert np.abs(o["xs"][st] - mean).max() <= 1e-11 * max(1.0, np.abs(mean).max())
        assert np.abs(o["Ps"][st] - dcov).max() <= 1e-11 * max(1.0, np.abs(dcov).max())


def _later_likelihood(wl, s, k):
    """p(y_{k+1..T} | x_k) as a Gaussian in x_k (precision, precision * mean),
    by dense conditioning of the joint Gaussian; the prior drops out because
    the later measurements depend on the past only through x_k."""
    mu, Sx, Hb, Rb, rb = _dense.joint_gaussian(wl, s)
    nx, ny = wl.nx, wl.ny
    st = wl.seg_steps(s)
    yv = wl.y[:, st].T.reshape(-1)
    rows = slice(k * ny, None)
    Hl, Rl, rl, yl = Hb[rows], Rb[rows, rows], rb[rows], yv[rows]
    ks = slice(k * nx, (k + 1) * nx)
    Cxx = Sx[ks, ks]
    Cyx = Hl @ Sx[:, ks]
    Cyy = Hl @ Sx @ Hl.T + Rl
    G = np.linalg.solve(Cxx, Cyx.T).T
    delta = Hl @ mu + rl - G @ mu[ks]
    Sig = Cyy - G @ Cyx.T
    prec = G.T @ np.linalg.solve(Sig, G)
    info = G.T @ np.linalg.solve(Sig, yl - delta)
    return prec, info


@pytest.mark.parametrize("case", [0, 1, 2, 5])
def test_backward_filter_equals_later_measurement_likelihood(case):
    """The kappa -> infinity combination of Sec. 4.3: Cbar = A J^{-1} A^T + C,
    bbar = A J^{-1} eta + b (with the + b of the first element; the printed
    bbar_0 has no b_0) is the likelihood of the later measurements as a
    function of x_k, N(x_k; bbar, Cbar) up to a constant."""
    wl = _tf_cases()[case]
    o = cref.two_filter(wl, suffix=True)
    suf = o["suf"]
    T = wl.seg_off[1] - wl.seg_off[0]
    checked = 0
    for k in (0, T // 2, T - 3):
        A, b, C, eta, J = (suf[n][k] for n in ("A", "b", "C", "eta", "J"))
        assert np.linalg.cond(J) < 1e10
        Ji = np.linalg.inv(J)
        Cbar = A @ Ji @ A.T + C
        bbar = A @ Ji @ eta + b
        prec, info = _later_likelihood(wl, 0, k)
        Cd = np.linalg.inv(prec)
        bd = Cd @ info
        assert np.abs(Cbar - Cd).max() <= 1e-9 * np.abs(Cd).max()
        assert np.abs(bbar - bd).max() <= 1e-9 * max(1.0, np.abs(bd).max())
        checked += 1
    assert checked == 3


@pytest.mark.parametrize("case", [0, 2, 5])
def test_two_filter_joint_solve_equals_printed_formula(case):
    """Where the later run's J is invertible the oracle's joint minimisation
    equals eq. twofilter as printed: x = (I + Cbar S)^{-1} (bbar + Cbar v)
    with S = P^{-1}, v = P^{-1} m of the forward filter (Sec. 2.5)."""
    wl = _tf_cases()[case]
    o = cref.two_filter(wl, suffix=True)
    suf = o["suf"]
    nx = wl.nx
    n = 0
    for k in range(wl.n_states):
        J = suf["J"][k]
        if np.linalg.cond(J) > 1e8:
            continue
        Ji = np.linalg.inv(J)
        Cbar = suf["A"][k] @ Ji @ suf["A"][k].T + suf["C"][k]
        bbar = suf["A"][k] @ Ji @ suf["eta"][k] + suf["b"][k]
        S = np.linalg.inv(o["P"][k])
        v = S @ o["m"][k]
        x = np.linalg.solve(np.eye(nx) + Cbar @ S, bbar + Cbar @ v)
        assert np.abs(x - o["xs"][k]).max() <= 1e-9 * max(1.0, np.abs(x).max())
        n += 1
    assert n >= wl.n_states // 2


def test_two_filter_end_state_is_filter():
    """At a segment's last state the later run is empty (I, 0, 0, 0, 0) and the
    two-filter estimate is the filter's."""
    wl = _tf_cases()[3]
    o = cref.two_filter(wl, suffix=True)
    last = wl.n_states - 1
    assert np.array_equal(o["suf"]["A"][last], np.eye(wl.nx))
    assert not o["suf"]["J"][last].any() and not o["suf"]["C"][last].any()
    assert np.abs(o["xs"][last] - o["m"][last]).max() <= 1e-12 * np.abs(o["m"][last]).max()
    assert np.abs(o["Ps"][last] - o["P"][last]).max() <= 1e-12 * np.abs(o["P"][last]).max()


# ------------------------------------------------------------------ coordinated turn (Sec. 5.2)
from oracle import models as _models


def test_ct_drift_is_a_coordinated_turn():
    """With the turn rate held and no noise the drift moves the target on a
    circle at constant speed: velocity rotated by omega t, position
    p0 + (sin(w t) v0 + (1 - cos(w t)) J v0) / w with J the +90 degree rotation.
    RK4 on the oracle's drift against that closed form."""
    th = torch.tensor([5e-4, 0.02, 5e-3, 1e-3], dtype=torch.float64)
    x0 = torch.tensor([[5.0, 5.0, 0.2, 0.3, 0.35]], dtype=torch.float64)
    f = lambda x: _models.drift_torch("ct", th, x, 5)[0]
    h, n = 1e-3, 4000
    x = x0.clone()
    for _ in range(n):
        k1 = f(x); k2 = f(x + 0.5 * h * k1); k3 = f(x + 0.5 * h * k2); k4 = f(x + h * k3)
        x = x + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    t, w = n * h, 0.35
    v0 = np.array([0.2, 0.3])
    Jv0 = np.array([-0.3, 0.2])
    v = np.cos(w * t) * v0 + np.sin(w * t) * Jv0
    p = np.array([5.0, 5.0]) + (np.sin(w * t) * v0 + (1 - np.cos(w * t)) * Jv0) / w
    assert np.abs(x[0, :2].numpy() - p).max() < 1e-11
    assert np.abs(x[0, 2:4].numpy() - v).max() < 1e-11
    assert x[0, 4].item() == 0.35


def test_ct_measurement_at_known_points():
    th = torch.tensor([5e-4, 0.02, 5e-3, 1e-3], dtype=torch.float64)
    pts = torch.tensor([[3.0, 4.0, 0, 0, 0], [-1.0, 0.0, 0, 0, 0], [0.0, -2.0, 0, 0, 0],
                        [-1.0, -1.0, 0, 0, 0]], dtype=torch.float64)
    _, hx = _models.drift_torch("ct", th, pts, 5)
    want = np.array([[5.0, np.arctan(4.0 / 3.0)], [1.0, np.pi], [2.0, -np.pi / 2],
                     [np.sqrt(2.0), -3 * np.pi / 4]])
    assert np.abs(hx.numpy() - want).max() < 1e-15
    e = np.array([0.1, np.pi - 1e-9, -np.pi, np.pi, 7.0, -7.0])
    w = _models.wrap_angle(e)
    assert np.all(w >= -np.pi) and np.all(w < np.pi)
    assert np.abs(np.sin(w) - np.sin(e)).max() < 1e-14 and np.abs(np.cos(w) - np.cos(e)).max() < 1e-14


def test_ct_taylor_terms_match_finite_differences():
    """F = df/dx, H = dh/dx at xbar by central differences of the drift and
    measurement; c, r make the expansion exact at xbar."""
    rng = np.random.default_rng(3)
    xb = np.column_stack([rng.uniform(2, 8, 6), rng.uniform(-8, 8, 6), rng.normal(0, 0.5, 6),
                          rng.normal(0, 0.5, 6), rng.normal(0, 0.3, 6)])
    th = np.array([5e-4, 0.02, 5e-3, 1e-3])
    F, c, L, W, H, r, R = _models.terms_numpy("ct", th, xb, 5)
    tt = torch.tensor(th)

    def fh(x):
        f, hx = _models.drift_torch("ct", tt, torch.tensor(x), 5)
        return f.numpy(), hx.numpy()
    eps = 1e-6
    for j in range(5):
        dp = xb.copy(); dp[:, j] += eps
        dm = xb.copy(); dm[:, j] -= eps
        (fp, hp), (fm, hm) = fh(dp), fh(dm)
        assert np.abs((fp - fm) / (2 * eps) - F[:, :, j]).max() < 1e-8
        assert np.abs((hp - hm) / (2 * eps) - H[:, :, j]).max() < 1e-8
    f0, h0 = fh(xb)
    assert np.abs(np.einsum("kij,kj->ki", F, xb) + c - f0).max() < 1e-14
    assert np.abs(np.einsum("kij,kj->ki", H, xb) + r - h0).max() < 1e-13
    assert np.allclose(L @ W @ L.T, np.diag([0, 0, th[0] ** 2, th[0] ** 2, th[1] ** 2]))


def test_ct_bearing_shift_by_two_pi_changes_nothing():
    wl = workloads.ct(n_seg=2, T=300, seed=81)
    xb = np.ascontiguousarray(wl.x_true)
    a = cref.smooth(wl, xb)
    w2 = workloads.Workload(**{**wl.__dict__})
    w2.y = wl.y.copy()
    k = np.arange(0, w2.y.shape[1], 7)
    w2.y[1, k] += 2 * np.pi * np.where(k % 2 == 0, 1.0, -1.0)
    b = cref.smooth(w2, xb)
    for key in ("xs", "Ps", "m", "P"):
        assert np.abs(a[key] - b[key]).max() <= 1e-11 * np.abs(a[key]).max()
    assert np.abs(a["loglik"] - b["loglik"]).max() <= 1e-11 * np.abs(a["loglik"]).max()


def test_ct_gauss_newton_matches_constrained_least_squares():
    """Gauss--Newton (Sec. 4.4) on the coordinated-turn model converges to the
    minimiser of the nonlinear discretised objective.  Q is singular (the
    position rows of L are zero), so the least-squares problem is written in
    the free variables: x_0 and, per step, the velocity and turn rate; the
    positions follow from xi_k = xi_{k-1} + dt dxi_k (the noise-free rows of
    the implicit-Euler step)."""
    wl = workloads.ct(n_seg=1, T=40, dt=0.05, seed=82, n_iter=14)
    o = cref.iterate(wl)
    sv, sw, r1, r2 = wl.theta[0]
    T, dt = wl.n_steps, wl.dt[0]
    y = wl.y
    P0i = np.linalg.cholesky(np.linalg.inv(wl.P0[0])).T

    def states(z):
        x0 = z[:5]
        vw = z[5:].reshape(T, 3)
        pos = x0[:2] + dt * np.cumsum(vw[:, :2], 0)
        xs = np.column_stack([pos, vw])
        return np.vstack([x0, xs])

    def resid(z):
        x = states(z)
        v, om = x[:, 2:4], x[:, 4]
        fv = np.column_stack([-om[1:] * v[1:, 1], om[1:] * v[1:, 0]])
        Dv = (v[1:] - v[:-1] - dt * fv) / (np.sqrt(dt) * sv)
        Dw = (om[1:] - om[:-1]) / (np.sqrt(dt) * sw)
        hr = np.hypot(x[1:, 0], x[1:, 1])
        hb = np.arctan2(x[1:, 1], x[1:, 0])
        eb = y[1] - hb
        eb = eb - 2 * np.pi * np.floor(eb / (2 * np.pi) + 0.5)
        E = np.concatenate([(y[0] - hr) * np.sqrt(dt / r1), eb * np.sqrt(dt / r2)])
        return np.concatenate([P0i @ (x[0] - wl.m0[0]), Dv.reshape(-1), Dw, E])

    xg = o["xs"]
    z0 = np.concatenate([xg[0], xg[1:, 2:].reshape(-1)])
    sol = scipy.optimize.least_squares(resid, z0 + 1e-3, xtol=1e-15, ftol=1e-15, gtol=1e-15)
    x_ls = states(sol.x)
    assert np.abs(xg - x_ls).max() < 1e-7 * np.abs(x_ls).max()
    # the positions of the Gauss--Newton solution obey the noise-free rows
    assert np.abs(xg[1:, :2] - xg[:-1, :2] - dt * xg[1:, 2:4]).max() < 1e-12


def test_ct_iterates_c_and_torch_agree_and_decrease():
    wl = workloads.ct(n_seg=2, T=150, dt=0.02, seed=83, n_iter=5)
    o = cref.iterate(wl, keep_iterates=True)
    for s in range(2):
        seg = ref.workload_segment(wl, s)
        its, _ = ref.gauss_newton("ct", seg["theta"], seg["dt"], seg["y"], seg["m0"], seg["P0"],
                                  5, 5)
        st = wl.seg_states(s)
        for i in range(5):
            np.testing.assert_allclose(o["iterates"][i][:, st].T, its[i].numpy(), rtol=0,
                                       atol=1e-9 * np.abs(its[i].numpy()).max())
        obj = [ref.map_objective_nonlinear("ct", seg["theta"], x, seg["dt"], seg["y"], seg["m0"],
                                           seg["P0"], 5).item() for x in its]
        assert all(b <= a + 1e-9 * abs(a) for a, b in zip(obj[1:], obj[2:]))


def test_zero_step_segments():
    """A segment without steps is its prior alone: x* = m0, P^s = P0, zero
    log-likelihood and objective; its neighbours are unaffected (dense
    conditioning per segment), in the RTS and the two-filter forms."""
    wl = workloads.cv_batched(lens=[0, 5, 0, 0, 30, 0], d=2, dt=0.05, seed=41)
    o = cref.smooth(wl)
    t = cref.two_filter(wl)
    for s in range(wl.n_seg):
        st = wl.seg_states(s)
        if wl.seg_off[s + 1] == wl.seg_off[s]:
            for out in (o, t):
                assert np.array_equal(out["xs"][st][0], wl.m0[s])
                assert np.abs(out["Ps"][st][0] - wl.P0[s]).max() < 1e-15
            assert o["loglik"][s] == 0.0 and o["mstar"][s] == 0.0
            continue
        mean, cov, ll = _dense.dense_posterior(wl, s)
        for out in (o, t):
            assert np.abs(out["xs"][st] - mean).max() <= 1e-11 * np.abs(mean).max()
        assert abs(o["loglik"][s] - ll) <= 1e-10 * abs(ll)


# ------------------------------------------------------------------ sub-stepped block elements
def test_substep_euler_block_converges_to_the_exact_block_with_corrected_sign():
    """Sub-stepped blocks (the paper's T blocks x n Euler substeps): over a
    block of fixed length, the Euler-integrated element ODE approaches the
    exact combination of the n one-step elements (the oracle's run over the
    block's steps, Sec. 4.1 rule) at first order in the substep with the
    A equation read as +A Q J, and stays O(1) away with the printed sign."""
    rng = np.random.default_rng(5)
    nx, ny = 3, 2
    F = rng.normal(0, 0.6, (nx, nx))
    c = rng.normal(0, 0.5, nx)
    L = rng.normal(0, 1.0, (nx, nx))
    Q = L @ L.T
    H = rng.normal(0, 1.0, (ny, nx))
    R = np.diag([0.3, 0.5])
    r = rng.normal(0, 0.2, ny)
    Tb = 0.8
    errs, errs_printed = [], []
    for n in (20, 40, 80, 160):
        h = Tb / n
        ts = h * np.arange(1, n + 1)
        ys = np.stack([np.sin(1.3 * ts + 0.2), np.cos(0.7 * ts)], 1)
        # the oracle's run of these n steps: the run after state 0 of an
        # n-step segment (a linear model with these constant terms)
        wl = workloads.linear_random(T=n, nx=nx, ny=ny, nw=nx, dt=h, time_varying=False, seed=1)
        wl.lin = dict(F=F, c=c, L=L, W=np.eye(nx), H=H, r=r, R=R)
        wl.lin = {k: (np.broadcast_to(v, (n,) + v.shape).copy() if k in ("F", "c", "H", "r") else v)
                  for k, v in wl.lin.items()}
        wl.y = ys.T.copy()
        o = cref.two_filter(wl, suffix=True)
        exact = [o["suf"][k][0] for k in ("A", "b", "C", "eta", "J")]
        for sign, out in ((+1.0, errs), (-1.0, errs_printed)):
            eu = oracle_blocks.euler_block(F, c, Q, H, np.linalg.inv(R), r, ys, h, sign)[-1]
            out.append(max(np.abs(e - x).max() / max(1.0, np.abs(x).max()) for e, x in zip(eu, exact)))
    ratios = [a / b for a, b in zip(errs[:-1], errs[1:])]
    assert all(1.8 < q < 2.2 for q in ratios), (errs, ratios)
    assert errs[-1] < 2e-2
    assert min(errs_printed) > 20 * errs[-1], (errs_printed, errs)


# ------------------------------------------------------------------ exact LTI discretisation
from oracle import lti as _lti


def test_van_loan_matches_constant_velocity_closed_forms():
    """Wiener velocity: Phi = [[1, dt], [0, 1]], Qd = q [[dt^3/3, dt^2/2], [dt^2/2, dt]];
    damped velocity (Ornstein-Uhlenbeck) with its integral: the classical formulas."""
    q, dt = 0.7, 0.05
    F = np.array([[0.0, 1.0], [0.0, 0.0]])
    L = np.array([[0.0], [1.0]])
    Phi, u, Qd = _lti.van_loan(F, np.zeros(2), L, q * np.eye(1), dt)
    assert np.abs(Phi - [[1, dt], [0, 1]]).max() < 1e-15
    assert np.abs(Qd - q * np.array([[dt ** 3 / 3, dt ** 2 / 2], [dt ** 2 / 2, dt]])).max() < 1e-16
    g = 0.8
    F = np.array([[0.0, 1.0], [0.0, -g]])
    Phi, u, Qd = _lti.van_loan(F, np.array([0.3, -0.2]), L, q * np.eye(1), dt)
    e = np.exp(-g * dt)
    assert np.abs(Phi - [[1, (1 - e) / g], [0, e]]).max() < 1e-15
    qvv = q * (1 - e * e) / (2 * g)
    qpv = q * (1 - e) ** 2 / (2 * g * g)
    qpp = q / g ** 2 * (dt - 2 * (1 - e) / g + (1 - e * e) / (2 * g))
    assert np.abs(Qd - [[qpp, qpv], [qpv, qvv]]).max() < 1e-15
    # u = int_0^dt e^{F s} ds c
    s = np.linspace(0, dt, 20001)
    integrand = np.stack([np.array([[1, (1 - np.exp(-g * t)) / g], [0, np.exp(-g * t)]]) @ [0.3, -0.2]
                          for t in s])
    assert np.abs(u - np.trapezoid(integrand, s, axis=0)).max() < 1e-11


def _exact_joint(wl, Fc, cc, Lc, Wc, H, r, R):
    """Dense joint Gaussian of (x_0..x_T) and y under the exact transitions."""
    T = wl.n_steps
    nx, ny = wl.nx, wl.ny
    dt = wl.dt[0]
    Phi, u, Qd = _lti.van_loan(Fc, cc, Lc, Wc, dt)
    n = (T + 1) * nx
    mu = np.zeros(n)
    mu[:nx] = wl.m0[0]
    G = np.zeros((n, n))
    G[:nx, :nx] = np.eye(nx)
    Cxi = np.zeros((n, n))
    Cxi[:nx, :nx] = wl.P0[0]
    for k in range(T):
        mu[(k + 1) * nx:(k + 2) * nx] = Phi @ mu[k * nx:(k + 1) * nx] + u
        G[(k + 1) * nx:(k + 2) * nx] = Phi @ G[k * nx:(k + 1) * nx]
        G[(k + 1) * nx:(k + 2) * nx, (k + 1) * nx:(k + 2) * nx] += np.eye(nx)
        Cxi[(k + 1) * nx:(k + 2) * nx, (k + 1) * nx:(k + 2) * nx] = Qd
    Sx = G @ Cxi @ G.T
    Hb = np.zeros((T * ny, n))
    Rb = np.zeros((T * ny, T * ny))
    for k in range(T):
        Hb[k * ny:(k + 1) * ny, (k + 1) * nx:(k + 2) * nx] = H
        Rb[k * ny:(k + 1) * ny, k * ny:(k + 1) * ny] = R / dt
    yv = wl.y.T.reshape(-1)
    my = Hb @ mu + np.tile(r, T)
    Sy = Hb @ Sx @ Hb.T + Rb
    K = np.linalg.solve(Sy, Hb @ Sx).T
    mean = mu + K @ (yv - my)
    cov = Sx - K @ Hb @ Sx
    return mean.reshape(T + 1, nx), cov


def lti_exact_workload(T=30, dt=0.08, seed=51, gamma=0.6):
    """A damped 2-D constant-velocity track with a drift offset, as a general
    linear workload whose terms are the exact discretisation's (oracle side)."""
    wl = workloads.cv(T=T, d=2, dt=dt, gamma=gamma, q=0.5, r=0.05, m0=[5, 5, 0, 0],
                      P0=1e-2 * np.eye(4), seed=seed)
    F = np.zeros((4, 4)); F[:2, 2:] = np.eye(2); F[2:, 2:] = -gamma * np.eye(2)
    c = np.array([0.0, 0.0, 0.15, -0.1])
    L = np.vstack([np.zeros((2, 2)), np.eye(2)])
    W = 0.5 * np.eye(2)
    H = np.hstack([np.eye(2), np.zeros((2, 2))])
    r = np.array([0.02, -0.03])
    R = 0.05 * np.eye(2)
    Ft, ct, Lt, Wt = _lti.implicit_equivalent(F, c, L, W, dt)
    # per-step arrays for F, c, H, r (the workloads' linear-model layout)
    per = lambda m: np.broadcast_to(m, (T,) + m.shape).copy()
    lin = dict(F=per(Ft), c=per(ct), L=Lt, W=Wt, H=per(H), r=per(r), R=R)
    w = workloads.Workload(name="lti_exact", model="linear", nx=4, ny=2, nw=4,
                           seg_off=wl.seg_off, dt=wl.dt, y=wl.y, theta=np.zeros((1, 0)),
                           m0=wl.m0, P0=wl.P0, x_true=wl.x_true, lin=lin)
    return w, (F, c, L, W, H, r, R)


def test_exact_discretisation_equals_dense_conditioning():
    """The oracle's filter and smoother on the implicit-equivalent terms give
    the posterior of the exactly discretised model (dense conditioning with
    Phi = e^{F dt}, Qd from scipy's expm written out here)."""
    wl, (F, c, L, W, H, r, R) = lti_exact_workload()
    o = cref.smooth(wl)
    mean, cov = _exact_joint(wl, F, c, L, W, H, r, R)
    nx = 4
    assert np.abs(o["xs"] - mean).max() <= 1e-11 * np.abs(mean).max()
    dcov = np.stack([cov[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(wl.n_steps + 1)])
    assert np.abs(o["Ps"] - dcov).max() <= 1e-11 * np.abs(dcov).max()


def test_implicit_euler_and_exact_agree_to_first_order():
    """Both discretisations approximate the same continuous-time problem: with
    one smooth measurement signal sampled on each grid, the smoothed means on a
    fixed horizon differ by O(dt)."""
    diffs = []
    for T in (40, 80, 160, 320):
        wl, (F, c, L, W, H, r, R) = lti_exact_workload(T=T, dt=3.2 / T, seed=52)
        t = wl.dt[0] * np.arange(1, T + 1)
        wl.y = np.stack([5 + 0.4 * np.sin(1.1 * t), 5 + 0.3 * np.cos(0.8 * t) + 0.2 * t])
        ex = cref.smooth(wl)["xs"]
        w2 = workloads.Workload(**{**wl.__dict__})
        per = lambda m: np.broadcast_to(m, (T,) + m.shape).copy()
        w2.lin = dict(F=per(F), c=per(c), L=L, W=W, H=per(H), r=per(r), R=R)
        w2.nw = 2
        ie = cref.smooth(w2)["xs"]
        diffs.append(np.abs(ex - ie).max())
    q = [a / b for a, b in zip(diffs[:-1], diffs[1:])]
    assert all(1.7 < x < 2.3 for x in q), (diffs, q)


# ------------------------------------------------------------------ Lorenz-63 terms
LORENZ_TH = np.array([10.0, 28.0, 8.0 / 3.0, 0.5, 0.5])


def test_lorenz_drift_fixed_points_divergence_and_symmetry():
    """The oracle's Lorenz-63 drift against properties of the system that do
    not come from its formula: it vanishes at the origin and at the two
    equilibria (+-sqrt(beta (rho - 1)), +-sqrt(beta (rho - 1)), rho - 1); its
    divergence, the trace of F, is the constant -(sigma + 1 + beta) (the
    divergence term of eq. OM is therefore constant for this model); and it is
    equivariant under (x1, x2, x3) -> (-x1, -x2, x3)."""
    sg, rho, be = LORENZ_TH[:3]
    a = np.sqrt(be * (rho - 1.0))
    eq = np.array([[0.0, 0.0, 0.0], [a, a, rho - 1.0], [-a, -a, rho - 1.0]])
    f, h = _models.drift_torch("lorenz63", torch.tensor(LORENZ_TH), torch.tensor(eq), 3)
    assert np.abs(f.numpy()).max() < 1e-12
    assert np.abs(h.numpy() - eq).max() == 0.0            # full-state measurement
    rng = np.random.default_rng(7)
    x = rng.normal(0, 8, (20, 3))
    for terms in (_models.terms_numpy, lambda *a: [t.numpy() for t in _models.terms_torch(
            a[0], torch.tensor(a[1]), torch.tensor(a[2]), a[3])]):
        F = np.asarray(terms("lorenz63", LORENZ_TH, x, 3)[0])
        assert np.abs(np.trace(F, axis1=1, axis2=2) + (sg + 1.0 + be)).max() < 1e-12
    P = np.diag([-1.0, -1.0, 1.0])
    fx, _ = _models.drift_torch("lorenz63", torch.tensor(LORENZ_TH), torch.tensor(x), 3)
    fpx, _ = _models.drift_torch("lorenz63", torch.tensor(LORENZ_TH), torch.tensor(x @ P), 3)
    assert np.abs(fpx.numpy() - fx.numpy() @ P).max() < 1e-12
    # the equilibria C+- are the only ones with x3 > 0: f(x) = 0 there fixes
    # x1 = x2 and x1^2 = beta x3, x3 = rho - 1 (a sign slip in any of the
    # three components moves one of them)
    assert np.abs(f.numpy()[1:, 2]).max() < 1e-12


@pytest.mark.parametrize("impl", ["numpy", "torch"])
def test_lorenz_taylor_terms_match_finite_differences(impl):
    """F = df/dx and H = dh/dx at xbar by central differences of the drift
    and measurement; c and r make the expansion exact at xbar (both the numpy
    terms, which feed the C oracle, and the torch terms, which give the
    gradient truth)."""
    rng = np.random.default_rng(4)
    xb = rng.normal(0, 8, (12, 3)) + np.array([0.0, 0.0, 20.0])
    th = LORENZ_TH.copy()
    if impl == "numpy":
        F, c, L, W, H, r, R = _models.terms_numpy("lorenz63", th, xb, 3)
    else:
        F, c, L, W, H, r, R = (t.numpy() for t in _models.terms_torch(
            "lorenz63", torch.tensor(th), torch.tensor(xb), 3))
    tt = torch.tensor(th)

    def fh(x):
        f, hx = _models.drift_torch("lorenz63", tt, torch.tensor(x), 3)
        return f.numpy(), hx.numpy()
    eps = 1e-5
    for j in range(3):
        dp = xb.copy(); dp[:, j] += eps
        dm = xb.copy(); dm[:, j] -= eps
        (fp, hp), (fm, hm) = fh(dp), fh(dm)
        # f is quadratic: the central difference is exact up to rounding
        assert np.abs((fp - fm) / (2 * eps) - F[:, :, j]).max() < 1e-7
        assert np.abs((hp - hm) / (2 * eps) - H[:, :, j]).max() < 1e-9
    f0, h0 = fh(xb)
    assert np.abs(np.einsum("kij,kj->ki", F, xb) + c - f0).max() < 1e-12
    assert np.abs(np.einsum("kij,kj->ki", H, xb) + r - h0).max() < 1e-12
    assert np.allclose(L @ W @ L.T, th[3] * np.eye(3)) and np.allclose(R, th[4] * np.eye(3))


def test_lorenz_terms_theta_dependence_matches_differences():
    """The theta dependence of the torch terms (which the oracle's autograd
    gradients differentiate) against central differences of the drift in
    theta: d(F xbar + c)/d theta = df/d theta at xbar, and d F / d theta equals
    the difference of F."""
    rng = np.random.default_rng(5)
    xb = torch.tensor(rng.normal(0, 8, (6, 3)))
    th = torch.tensor(LORENZ_TH).requires_grad_(True)
    F, c, L, W, H, r, R = _models.terms_torch("lorenz63", th, xb, 3)
    lin = torch.einsum("kij,kj->ki", F, xb) + c
    for k in range(6):
        for i in range(3):
            g, = torch.autograd.grad(lin[k, i], th, retain_graph=True)
            for t in range(3):
                e = 1e-6 * LORENZ_TH[t]
                tp, tm = LORENZ_TH.copy(), LORENZ_TH.copy()
                tp[t] += e
                tm[t] -= e
                fp, _ = _models.drift_torch("lorenz63", torch.tensor(tp), xb, 3)
                fm, _ = _models.drift_torch("lorenz63", torch.tensor(tm), xb, 3)
                fd = (fp[k, i] - fm[k, i]).item() / (2 * e)
                assert abs(g[t].item() - fd) < 1e-6 * max(1.0, abs(fd)), (k, i, t)
    for t in range(3):
        e = 1e-6 * LORENZ_TH[t]
        tp, tm = LORENZ_TH.copy(), LORENZ_TH.copy()
        tp[t] += e
        tm[t] -= e
        Fp = _models.terms_numpy("lorenz63", tp, xb.numpy(), 3)[0]
        Fm = _models.terms_numpy("lorenz63", tm, xb.numpy(), 3)[0]
        dF = np.zeros((3, 3))
        for a in range(3):
            for b in range(3):
                gab, = torch.autograd.grad(F[0, a, b], th, retain_graph=True, allow_unused=True)
                dF[a, b] = 0.0 if gab is None else gab[t].item()
        assert np.abs((Fp[0] - Fm[0]) / (2 * e) - dF).max() < 1e-6


def test_lorenz_gauss_newton_matches_nonlinear_least_squares():
    """Gauss--Newton (Sec. 4.4) on Lorenz-63 (Q = q I invertible) converges to
    the minimiser of the nonlinear discretised objective found by a generic
    trust-region least-squares solver on its stacked residuals (prior, the
    step residuals x_k - x_{k-1} - dt f(x_k) weighted by (dt q)^{-1/2}, the
    measurements weighted by (dt / r)^{1/2}); the objective decreases and is
    stationary at the last iterate."""
    wl = workloads.lorenz63(n_seg=1, T=40, dt=0.01, seed=72, n_iter=12)
    seg = ref.workload_segment(wl, 0)
    its, out = ref.gauss_newton("lorenz63", seg["theta"], seg["dt"], seg["y"], seg["m0"],
                                seg["P0"], 3, 12)
    obj = [ref.map_objective_nonlinear("lorenz63", seg["theta"], x, seg["dt"], seg["y"],
                                       seg["m0"], seg["P0"], 3).item() for x in its]
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(obj[2:], obj[3:]))
    q, rr = wl.theta[0][3], wl.theta[0][4]
    T = wl.n_steps
    dt = wl.dt[0]
    y = wl.y.T
    P0h = np.linalg.cholesky(np.linalg.inv(wl.P0[0])).T
    tt = torch.tensor(wl.theta[0])

    def resid(z):
        x = z.reshape(T + 1, 3)
        f, hx = _models.drift_torch("lorenz63", tt, torch.tensor(x[1:]), 3)
        D = (x[1:] - x[:-1] - dt * f.numpy()) / np.sqrt(dt * q)
        E = (y - hx.numpy()) * np.sqrt(dt / rr)
        return np.concatenate([P0h @ (x[0] - wl.m0[0]), D.reshape(-1), E.reshape(-1)])

    sol = scipy.optimize.least_squares(resid, its[-1].numpy().reshape(-1) + 0.05, xtol=1e-15,
                                       ftol=1e-15, gtol=1e-15)
    x_ls = sol.x.reshape(T + 1, 3)
    assert np.abs(its[-1].numpy() - x_ls).max() < 1e-7 * np.abs(x_ls).max()
    assert abs(0.5 * np.sum(resid(sol.x) ** 2) - obj[-1]) < 1e-9 * abs(obj[-1])
    x = its[-1].clone().requires_grad_(True)
    M = ref.map_objective_nonlinear("lorenz63", seg["theta"], x, seg["dt"], seg["y"],
                                    seg["m0"], seg["P0"], 3)
    g, = torch.autograd.grad(M, x)
    assert g.abs().max().item() < 1e-6


# ------------------------------------------------------------------ divergence term of eq. OM

@pytest.mark.parametrize("model", ["cv", "vdp", "lorenz63", "ct"])
def test_divergence_is_the_trace_of_the_drift_jacobian(model):
    """div f used by the Onsager--Machlup objective equals the trace of the
    drift's Jacobian by central differences of f itself."""
    from oracle import models
    nx = {"cv": 4, "vdp": 2, "lorenz63": 3, "ct": 5}[model]
    theta = torch.tensor({"cv": [0.3, 0.5, 0.05], "vdp": [1.5, 0.1, 0.05],
                          "lorenz63": [10.0, 28.0, 8.0 / 3.0, 0.5, 0.5],
                          "ct": [5e-4, 0.02, 5e-3, 1e-3]}[model], dtype=torch.float64)
    rng = np.random.default_rng(81)
    x = torch.tensor(rng.normal(0, 2, (7, nx)))
    div = models.divergence_torch(model, theta, x, nx)
    h = 1e-5
    tr = torch.zeros(7, dtype=torch.float64)
    for i in range(nx):
        e = torch.zeros(nx, dtype=torch.float64)
        e[i] = h
        fp, _ = models.drift_torch(model, theta, x + e, nx)
        fm, _ = models.drift_torch(model, theta, x - e, nx)
        tr += (fp[:, i] - fm[:, i]) / (2 * h)
    assert torch.allclose(div, tr, rtol=1e-8, atol=1e-8), (div, tr)


def test_om_newton_iteration_reaches_the_minimiser_of_the_om_objective():
    """Gauss--Newton on the energy part with a Newton step on the divergence
    term (Van der Pol, state-dependent divergence mu (1 - x1^2)) converges to
    the minimiser of the discretised Onsager--Machlup objective with its
    divergence term, found by a generic quasi-Newton minimiser; the objective
    decreases and its gradient vanishes there.  Without the term the iteration
    converges to a different point (the term matters)."""
    wl = workloads.vdp(T=40, dt=0.02, seed=82, n_iter=10)
    seg = ref.workload_segment(wl, 0)
    args = (seg["dt"], seg["y"], seg["m0"], seg["P0"], 2)
    its, out = ref.gauss_newton("vdp", seg["theta"], *args, 10, om_div=True)
    obj = [ref.om_objective("vdp", seg["theta"], x, *args).item() for x in its]
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(obj[1:], obj[2:])), obj
    x = its[-1].clone().requires_grad_(True)
    g, = torch.autograd.grad(ref.om_objective("vdp", seg["theta"], x, *args), x)
    assert g.abs().max().item() < 1e-8, g.abs().max()

    def fun(z):
        t = torch.tensor(z.reshape(-1, 2), requires_grad=True)
        val = ref.om_objective("vdp", seg["theta"], t, *args)
        gr, = torch.autograd.grad(val, t)
        return val.item(), gr.numpy().ravel()
    res = scipy.optimize.minimize(fun, its[0].numpy().ravel(), jac=True, method="BFGS",
                                  options={"gtol": 1e-11, "maxiter": 20000})
    xm = res.x.reshape(-1, 2)
    assert np.abs(xm - its[-1].numpy()).max() <= 1e-6 * np.abs(xm).max(), \
        np.abs(xm - its[-1].numpy()).max()
    its0, _ = ref.gauss_newton("vdp", seg["theta"], *args, 10, om_div=False)
    assert np.abs(its0[-1].numpy() - its[-1].numpy()).max() > 1e-4


# ------------------------------------------------------------------ sub-stepped blocks

@pytest.mark.parametrize("kind", ["cv", "vdp"])
def test_blocks_of_one_substep_are_the_kalman_filter_and_rts_smoother(kind):
    """With one substep per block the Euler element is the one-step element,
    and the block oracle's conditioning on backward transitions (covariance
    form with (P + C)^-1) reproduces the covariance Kalman filter and the RTS
    smoother of the discrete model (the pinned oracle) to rounding."""
    if kind == "cv":
        wl = workloads.cv_batched(lens=[40, 1, 25], seed=91, gamma=0.3)
        xbar = None
    else:
        wl = workloads.vdp(T=60, dt=0.02, seed=92, n_iter=2)
        xbar = cref.iterate(wl, n_iter=1)["xs"].T.copy()
    wb = workloads.blocks(wl, 1)
    o = cref.smooth(wl, xbar)
    b = oracle_blocks.smooth(wb, xbar)
    for k in ("m", "P", "xs", "Ps"):
        assert np.abs(b[k] - o[k]).max() <= 1e-11 * np.abs(o[k]).max(), k


def test_block_dense_output_converges_to_the_fine_grid_smoother():
    """Blocks of n = 4 Euler substeps with their dense output, on a smooth
    measurement signal over a fixed horizon: as the substep halves, the MAP
    states at the block boundaries and at the interior substeps (and the
    filter there) approach the smoother of the same problem on the fine grid
    (one exact element per substep: the pinned oracle) at least at first
    order (with blocks of fixed substep count the observed order is two: the
    error ratio per halving is about 4)."""
    errs, errs_f = [], []
    for T in (40, 80, 160):
        n = 4
        wl = workloads.cv(T=T * n, d=2, t_end=2.0, gamma=0.4, q=0.5, r=0.05,
                          m0=[1, 0, 0, 1], P0=0.1 * np.eye(4), seed=93)
        t = np.cumsum(wl.dt)
        wl.y = np.stack([np.sin(1.7 * t), np.cos(1.1 * t + 0.3)])
        o = cref.smooth(wl)
        b = oracle_blocks.smooth(workloads.blocks(wl, n))
        # dense states of block k (ending at block state k): fine states (k-1)*n + j
        d = np.zeros_like(o["xs"])
        d[::n] = b["xs"]
        for k in range(1, T + 1):
            for j in range(1, n):
                d[(k - 1) * n + j] = b["dense_xs"][k, j - 1]
        errs.append(np.abs(d - o["xs"]).max() / np.abs(o["xs"]).max())
        mf = np.zeros_like(o["m"])
        mf[::n] = b["m"]
        for k in range(1, T + 1):
            for j in range(1, n):
                mf[(k - 1) * n + j] = b["dense_m"][k, j - 1]
        errs_f.append(np.abs(mf - o["m"]).max() / np.abs(o["m"]).max())
    for e in (errs, errs_f):
        ratios = [a / c for a, c in zip(e[:-1], e[1:])]
        assert all(q > 1.7 for q in ratios), (e, ratios)
    assert errs[-1] < 1e-3 and errs_f[-1] < 1e-3, (errs, errs_f)
