"""Gradient parity on the GPU: map_backward, the implicit-function VJP of a
cotangent on x*, the MapSmooth autograd.Function, FP32 storage, and the timed
workloads (cfg2 at T = 2^20, cfg4's 4096 segments) against the oracle.

Metric, per gradient component i (and per segment):
    |g_i - ref_i| <= tol * max(|ref_i|, floor),  floor = f * max_j |ref_j|
over the components j of the same gradient vector.  FP64 storage: tol = 1e-6,
f = 1e-3: a component within a factor 1000 of the largest is held to 1e-6 of
itself, a smaller one (a derivative that vanishes by symmetry, e.g. d/dgamma
at gamma = 0) to 1e-9 of the largest.  FP32 storage (the FP32 run and the
FP64 oracle see the same FP32-rounded inputs): tol = 3e-4, f = 0.1.  A
gradient is a sum of one term per step built from the costates
lam = S (m - x*) (and nu = S (m' - mu) for the trajectory VJP), differences
of means that the FP32 planes round to eps32 of their size, so each term
carries eps32 |x| / |m - x*| and components whose terms cancel over the
horizon carry it relative to the terms, not to the sum: at T = 2^20,
d loglik/dq sums terms of order one to -2.09 and is within 1.2e-3 of itself
(2.3e-6 of the largest component, d loglik/dr), and the trajectory VJP's
largest component is within 1.4e-4.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref, ref
from tests.test_gpu_fullsize import sub_workload

pytestmark = pytest.mark.gpu

TORCH_DT = {"f64": torch.float64, "f32": torch.float32}
GTOL = {"f64": 1e-6, "f32": 3e-4}
FLOOR = {"f64": 1e-3, "f32": 0.1}


def grad_err(g, r, dtype="f64"):
    """max over components of |g_i - r_i| / max(|r_i|, f max_j |r_j|); the
    last axis indexes the components of one gradient vector."""
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    floor = FLOOR[dtype] * np.abs(r).max(axis=-1, keepdims=True)
    den = np.maximum(np.maximum(np.abs(r), floor), 1e-300)
    return float((np.abs(g - r) / den).max())


def _case(model, dtype="f64"):
    """A small workload, its oracle linearisation point (nonlinear models:
    the one of the last Gauss-Newton solve) and a device Problem set to it."""
    import paper_2512_13319_amd as ms
    if model == "cv":
        wl = workloads.cv_batched(n_seg=6, lmin=5.0, lmax=9.5, seed=71, gamma=0.25)
    elif model == "vdp":
        wl = workloads.vdp(T=400, dt=0.01, seed=72, n_iter=3)
    elif model == "lorenz63":
        wl = workloads.lorenz63(n_seg=3, T=250, dt=0.005, seed=73, n_iter=2)
    else:
        wl = workloads.ct(n_seg=2, T=300, seed=74, n_iter=2)
    wl = wl.rounded(dtype)
    xbar = None
    if model != "cv":
        xbar = cref.iterate(wl)["xbar"]
        if dtype == "f32":
            xbar = xbar.astype(np.float32).astype(np.float64)  # as the device stores it
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype],
                                 xbar=None if xbar is None else torch.tensor(xbar))
    return wl, xbar, p


def _seg_xbar(wl, xbar, s):
    st = wl.seg_states(s)
    if xbar is None:
        return torch.zeros(st.stop - st.start, wl.nx, dtype=torch.float64)
    return torch.tensor(xbar[:, st].T.copy())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", ["cv", "lorenz63", "ct"])
def test_backward_equals_fused_adjoint(model, dtype):
    """map_backward from the saved filter planes recomputes x*, P^s, the
    objective and both gradients as the fused map_smooth does: to rounding in
    FP64; with FP32 storage the recomputed trajectory maps start from the
    stored (rounded) S and mean where the fused pass had them in registers,
    so the two agree to the FP32 bar."""
    import paper_2512_13319_amd as ms
    from tests.test_gpu_parity import rel_err
    wl, xbar, p = _case(model, dtype)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False)
    b = ms.backward(p, r["S"], r["v"], covariances=True, objective=True, natural=False)
    torch.cuda.synchronize()
    tol = 1e-11 if dtype == "f64" else 1e-4
    for k, comps in (("xs", p.nx), ("Ps", p.nsym)):
        a = p.natural(b[k], comps).double().cpu().numpy().T
        c = p.natural(r[k], comps).double().cpu().numpy().T
        e = rel_err(a, c)
        print(f"{model} {dtype} backward vs fused {k}: {e:.1e}")
        assert e <= tol, k
    for k in ("obj", "g_loglik", "g_obj"):
        a, c = b[k].cpu().numpy(), r[k].cpu().numpy()
        e = grad_err(a, c, dtype)
        print(f"{model} {dtype} backward vs fused {k}: {e:.1e}")
        assert e <= tol, (k, a, c)


@pytest.mark.parametrize("model", ["cv", "vdp", "lorenz63", "ct"])
def test_trajectory_vjp_matches_oracle_autograd(model):
    """The implicit-function VJP: d(sum_k w_k . x*_k)/dtheta for a random w
    against autograd of the sequential oracle (linearisation point fixed),
    every segment, FP64."""
    import paper_2512_13319_amd as ms
    wl, xbar, p = _case(model)
    rng = np.random.default_rng(75)
    w = rng.normal(size=(wl.nx, wl.n_states))
    r = ms.smooth(p, covariances=False, loglik=False, objective=False, natural=False)
    b = ms.backward(p, r["S"], r["v"], covariances=False, objective=False, loglik_grad=False,
                    obj_grad=False, g_xs=torch.tensor(w))
    torch.cuda.synchronize()
    gx = b["g_xs_theta"].cpu().numpy()
    for s in range(wl.n_seg):
        seg = ref.workload_segment(wl, s)
        st = wl.seg_states(s)
        g = ref.trajectory_vjp(wl.model, wl.nx, seg, _seg_xbar(wl, xbar, s),
                               torch.tensor(w[:, st].T.copy())).numpy()
        e = grad_err(gx[s], g)
        print(f"{model} segment {s}: gpu {gx[s]} oracle {g} err {e:.1e}")
        assert e <= GTOL["f64"], (s, gx[s], g)


@pytest.mark.parametrize("shape", ["shared", "shared_row", "per_segment"])
def test_mapsmooth_autograd(shape):
    """torch.autograd through MapSmooth (cotangents on the log-likelihood, the
    objective and x*) equals the oracle's gradient of the same scalar; theta
    shared ([n_theta] or [1, n_theta]: gradients summed over segments) or per
    segment."""
    import paper_2512_13319_amd as ms
    wl, _, p = _case("cv")
    th0 = torch.tensor(wl.theta, dtype=torch.float64)
    if shape == "shared":
        theta = th0[0].clone()
        wl.theta = np.repeat(wl.theta[:1], wl.n_seg, axis=0)
    elif shape == "shared_row":
        theta = th0[:1].clone()
        wl.theta = np.repeat(wl.theta[:1], wl.n_seg, axis=0)
    else:
        theta = th0.clone()
    theta = theta.to("cuda").requires_grad_(True)
    rng = np.random.default_rng(76)
    w = rng.normal(size=(wl.nx, wl.n_states))
    xs, ll, obj = ms.MapSmooth.apply(theta, p)
    loss = 0.7 * ll.sum() - 1.3 * obj.sum() + (xs * torch.tensor(w, device="cuda")).sum()
    g, = torch.autograd.grad(loss, theta)
    g = g.cpu().numpy().reshape(-1, 3)
    ref_g = []
    for s in range(wl.n_seg):
        seg = ref.workload_segment(wl, s)
        st = wl.seg_states(s)
        xb = torch.zeros(st.stop - st.start, 4, dtype=torch.float64)
        gl, gm, _ = ref.gradients("cv", 4, seg, xb)
        gx = ref.trajectory_vjp("cv", 4, seg, xb, torch.tensor(w[:, st].T.copy()))
        ref_g.append((0.7 * gl - 1.3 * gm + gx).numpy())
    ref_g = np.stack(ref_g)
    if shape != "per_segment":
        ref_g = ref_g.sum(0, keepdims=True)
    e = grad_err(g, ref_g)
    print(f"MapSmooth {shape}: {g} vs {ref_g} err {e:.1e}")
    assert e <= GTOL["f64"]


@pytest.mark.parametrize("model", ["cv", "lorenz63"])
def test_fp32_storage_gradients(model):
    """FP32 storage (FP64 arithmetic): Fisher and envelope gradients and the
    trajectory VJP against oracle autograd on the same FP32-rounded inputs."""
    import paper_2512_13319_amd as ms
    wl, xbar, p = _case(model, "f32")
    rng = np.random.default_rng(77)
    w = rng.normal(size=(wl.nx, wl.n_states))
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False)
    b = ms.backward(p, r["S"], r["v"], covariances=False, objective=False, loglik_grad=False,
                    obj_grad=False, g_xs=torch.tensor(w))
    torch.cuda.synchronize()
    for s in range(wl.n_seg):
        seg = ref.workload_segment(wl, s)
        st = wl.seg_states(s)
        xb = _seg_xbar(wl, xbar, s)
        gl, gm, _ = ref.gradients(wl.model, wl.nx, seg, xb)
        gx = ref.trajectory_vjp(wl.model, wl.nx, seg, xb, torch.tensor(w[:, st].T.copy()))
        errs = [grad_err(r["g_loglik"][s].cpu().numpy(), gl.numpy(), "f32"),
                grad_err(r["g_obj"][s].cpu().numpy(), gm.numpy(), "f32"),
                grad_err(b["g_xs_theta"][s].cpu().numpy(), gx.numpy(), "f32")]
        print(f"{model} f32 segment {s}: loglik {errs[0]:.1e} obj {errs[1]:.1e} "
              f"vjp {errs[2]:.1e}")
        assert max(errs) <= GTOL["f32"]


def _step(th_i):
    """Five-point step for theta_i: 1e-3 |theta_i| (truncation error ~1e-12
    relative), 1e-3 where theta_i = 0 (gamma of the constant-velocity
    workloads)."""
    a = np.abs(th_i)
    return np.where(a > 0, 1e-3 * a, 1e-3)


def _five_point(wl_one, th, i, h, fn):
    vals = {}
    for k in (-2, -1, 1, 2):
        w = workloads.Workload(**{**wl_one.__dict__})
        w.theta = wl_one.theta.copy()
        w.theta[:, i] = th[:, i] + k * h
        vals[k] = fn(w)
    return (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cfg2_gradients_full_size(dtype):
    """The timed workload (T = 2^20, one trajectory): d loglik/dtheta,
    d M*/dtheta and the trajectory VJP of w (nonzero on 64 sampled states)
    against a five-point central difference of the C oracle (12 solves of
    2^20 steps)."""
    import paper_2512_13319_amd as ms
    wl = workloads.config(2).rounded(dtype)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype])
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False)
    rng = np.random.default_rng(78)
    w = np.zeros((4, wl.n_states))
    idx = np.unique(np.concatenate([[0, wl.n_states - 1], rng.choice(wl.n_states, 62)]))
    w[:, idx] = rng.normal(size=(4, idx.size))
    b = ms.backward(p, r["S"], r["v"], covariances=False, objective=False, loglik_grad=False,
                    obj_grad=False, g_xs=torch.tensor(w))
    torch.cuda.synchronize()
    th = wl.theta.copy()

    def f(wk):
        o = cref.smooth(wk)
        return np.array([o["loglik"][0], o["mstar"][0], (o["xs"].T * w).sum()])
    fd = np.stack([_five_point(wl, th, i, float(_step(th[0, i])), f) for i in range(3)])
    gl = r["g_loglik"][0].cpu().numpy()
    gm = r["g_obj"][0].cpu().numpy()
    gx = b["g_xs_theta"][0].cpu().numpy()
    tol = GTOL[dtype]
    for name, g, ref_g in (("loglik", gl, fd[:, 0]), ("obj", gm, fd[:, 1]), ("vjp", gx, fd[:, 2])):
        e = grad_err(g, ref_g, dtype)
        print(f"cfg2 {dtype} {name}: gpu {g} fd {ref_g} err {e:.1e}")
        assert e <= tol, name


def test_cfg4_sampled_gradients():
    """cfg4 in full (4096 segments, FP32 storage, the fused adjoint as timed):
    per-segment gradients of 16 sampled segments (shortest and longest
    included) against a five-point difference of the C oracle on those
    segments (each segment's values depend only on its own theta, so one
    perturbation of all sampled thetas serves them all)."""
    import paper_2512_13319_amd as ms
    wl = workloads.config(4).rounded("f32")
    lens = np.diff(wl.seg_off)
    rng = np.random.default_rng(79)
    segs = np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens)],
                                     rng.choice(wl.n_seg, 14, replace=False)]))
    p = ms.problem_from_workload(wl, dtype=torch.float32)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True)
    torch.cuda.synchronize()
    sub, _ = sub_workload(wl, segs)
    th = sub.theta.copy()

    def f(wk):
        o = cref.smooth(wk)
        return np.stack([o["loglik"], o["mstar"]])        # [2, n_sub]
    fd = np.stack([_five_point(sub, th, i, _step(th[:, i]), f) for i in range(3)])  # [3, 2, n_sub]
    gl = r["g_loglik"].cpu().numpy()[segs]
    gm = r["g_obj"].cpu().numpy()[segs]
    el = grad_err(gl, fd[:, 0, :].T, "f32")
    em = grad_err(gm, fd[:, 1, :].T, "f32")
    print(f"cfg4 f32 ({len(segs)} sampled segments): g_loglik {el:.1e} g_obj {em:.1e}")
    assert el <= GTOL["f32"] and em <= GTOL["f32"]
