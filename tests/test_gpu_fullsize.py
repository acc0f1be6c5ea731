"""Parity at the full workload sizes.

cfg2 (T = 2^20) and cfg3 (T = 2^18, 10 Gauss-Newton iterations) are compared
state by state against the C oracle.  cfg4 (4096 ragged segments, ~1.6e7
steps) and cfg5 (256 Lorenz-63 trajectories of 2^14 steps, 5 iterations) run
in full on the GPU; segments are independent, so the oracle recomputes a
sample of them (always including the shortest and the longest) and those
are compared one by one.  cfg5 gradients are checked against five-point central
differences of the oracle's log-likelihood and objective with the
linearisation point held fixed.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref, ref

pytestmark = pytest.mark.gpu

TORCH_DT = {"f64": torch.float64, "f32": torch.float32}
TOL = {"f64": 1e-9, "f32": 1e-4}


def rel_err(g, r):
    g = np.asarray(g, dtype=np.float64).reshape(g.shape[0], -1)
    r = np.asarray(r, dtype=np.float64).reshape(r.shape[0], -1)
    return float((np.abs(g - r).max(0) / np.maximum(np.abs(r).max(0), 1e-300)).max())


def sub_workload(wl, segs):
    """The listed segments of a workload as a workload of their own."""
    segs = np.asarray(segs)
    lens = wl.seg_off[segs + 1] - wl.seg_off[segs]
    so = np.zeros(len(segs) + 1, dtype=np.int64)
    so[1:] = np.cumsum(lens)
    st = np.concatenate([np.arange(wl.seg_off[s], wl.seg_off[s + 1]) for s in segs])
    xs = np.concatenate([np.arange(wl.seg_off[s] + s, wl.seg_off[s + 1] + s + 1) for s in segs])
    w = workloads.Workload(**{**wl.__dict__})
    w.seg_off, w.dt, w.y = so, wl.dt[st], wl.y[:, st]
    w.theta, w.m0, w.P0 = wl.theta[segs], wl.m0[segs], wl.P0[segs]
    w.x_true = wl.x_true[:, xs]
    return w, xs


def state_rows(wl, segs):
    return np.concatenate([np.arange(wl.seg_off[s] + s, wl.seg_off[s + 1] + s + 1) for s in segs])


def sym_full(ms, planes, nx):
    return ms.sym_to_full(planes, nx).double().cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cfg2_full(dtype):
    import paper_2512_13319_amd as ms
    wl = workloads.config(2).rounded(dtype)
    o = cref.smooth(wl)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype])
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True)
    torch.cuda.synchronize()
    e_xs = rel_err(r["xs"].cpu().numpy().T, o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"], 4), o["Ps"])
    e_ll = abs(r["loglik"].item() - o["loglik"][0]) / abs(o["loglik"][0])
    e_ob = abs(r["obj"].item() - o["mstar"][0]) / abs(o["mstar"][0])
    print(f"cfg2 {dtype}: xs {e_xs:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e} obj {e_ob:.2e}")
    tol = TOL[dtype]
    assert e_xs <= tol and e_Ps <= tol and e_ll <= tol and e_ob <= tol
    assert torch.isfinite(r["g_loglik"]).all() and torch.isfinite(r["g_obj"]).all()


def test_cfg3_full_vdp():
    import paper_2512_13319_amd as ms
    wl = workloads.config(3)
    o = cref.iterate(wl)
    p = ms.problem_from_workload(wl, dtype=torch.float64)
    r = ms.iterated_nonlinear(p, wl.n_iter, covariances=True, loglik=True, objective=True)
    torch.cuda.synchronize()
    e_xs = rel_err(r["xs"].cpu().numpy().T, o["xs"])
    e_xb = rel_err(r["xbar"].cpu().numpy().T, o["xbar"].T)
    e_Ps = rel_err(sym_full(ms, r["Ps"], 2), o["Ps"])
    e_ll = abs(r["loglik"].item() - o["loglik"][0]) / abs(o["loglik"][0])
    print(f"cfg3: xs {e_xs:.2e} xbar {e_xb:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e}")
    assert max(e_xs, e_xb, e_Ps, e_ll) <= 1e-9


def test_cfg4_full_batched_f32():
    import paper_2512_13319_amd as ms
    wl = workloads.config(4).rounded("f32")
    lens = np.diff(wl.seg_off)
    rng = np.random.default_rng(0)
    segs = np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens), 0, wl.n_seg - 1],
                                     rng.choice(wl.n_seg, 60, replace=False)]))
    sub, _ = sub_workload(wl, segs)
    o = cref.smooth(sub)
    p = ms.problem_from_workload(wl, dtype=torch.float32)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True)
    torch.cuda.synchronize()
    rows = state_rows(wl, segs)
    xs = r["xs"].cpu().numpy().T[rows]
    Ps = sym_full(ms, r["Ps"][:, torch.as_tensor(rows, device=r["Ps"].device)], 4)
    e_xs = rel_err(xs, o["xs"])
    e_Ps = rel_err(Ps, o["Ps"])
    ll = r["loglik"].cpu().numpy()[segs]
    ob = r["obj"].cpu().numpy()[segs]
    e_ll = np.max(np.abs(ll - o["loglik"]) / np.abs(o["loglik"]))
    e_ob = np.max(np.abs(ob - o["mstar"]) / np.abs(o["mstar"]))
    print(f"cfg4 f32 ({len(segs)} sampled segments): xs {e_xs:.2e} Ps {e_Ps:.2e} "
          f"ll {e_ll:.2e} obj {e_ob:.2e}")
    assert max(e_xs, e_Ps, e_ll, e_ob) <= 1e-4


def test_batched_f64_more_wavefronts_than_simds():
    """600 ragged constant-velocity tracks (~1.9e6 steps) in FP64 at 16 states
    per lane: the grid has more wavefronts than the chip has SIMDs, so the
    filter up-sweep runs its two-wavefront variant (which no single 2^20-step
    track reaches); the fused fix-up runs two wavefronts per SIMD at every
    size.  Sampled segments against the oracle at 1e-9, gradients within the
    per-component metric of tests/test_gpu_gradients.py."""
    import paper_2512_13319_amd as ms
    from tests.test_gpu_gradients import GTOL, grad_err
    wl = workloads.cv_batched(n_seg=600, lmin=11.0, lmax=12.0, seed=41, gamma=0.1)
    assert wl.n_steps + wl.n_seg > 1024 * 64 * 16  # more lanes than one wavefront per SIMD
    lens = np.diff(wl.seg_off)
    rng = np.random.default_rng(1)
    segs = np.unique(np.concatenate([[np.argmin(lens), np.argmax(lens), 0, wl.n_seg - 1],
                                     rng.choice(wl.n_seg, 12, replace=False)]))
    sub, _ = sub_workload(wl, segs)
    o = cref.smooth(sub)
    p = ms.problem_from_workload(wl, dtype=torch.float64, chunk=16)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True)
    torch.cuda.synchronize()
    rows = state_rows(wl, segs)
    e_xs = rel_err(r["xs"].cpu().numpy().T[rows], o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"][:, torch.as_tensor(rows, device=r["Ps"].device)], 4),
                   o["Ps"])
    ll = r["loglik"].cpu().numpy()[segs]
    ob = r["obj"].cpu().numpy()[segs]
    e_ll = np.max(np.abs(ll - o["loglik"]) / np.abs(o["loglik"]))
    e_ob = np.max(np.abs(ob - o["mstar"]) / np.abs(o["mstar"]))
    print(f"batched f64 ({len(segs)} sampled segments): xs {e_xs:.2e} Ps {e_Ps:.2e} "
          f"ll {e_ll:.2e} obj {e_ob:.2e}")
    assert max(e_xs, e_Ps, e_ll, e_ob) <= 1e-9
    # gradients of two sampled segments against oracle autograd
    for s in segs[:2]:
        seg = ref.workload_segment(wl, int(s))
        T = seg["y"].shape[0]
        gl, gm, _ = ref.gradients("cv", wl.nx, seg, torch.zeros(T + 1, wl.nx,
                                                                   dtype=torch.float64))
        for got, want in ((r["g_loglik"][s], gl), (r["g_obj"][s], gm)):
            assert grad_err(got.cpu().numpy(), want.numpy()) <= GTOL["f64"], (s, got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cfg5_full_lorenz_with_gradients(dtype):
    """256 Lorenz-63 trajectories of 2^14 steps, 5 Gauss-Newton iterations, in
    full on the GPU (FP64 or FP32 storage); three sampled trajectories against
    the oracle's iterations (FP32: on the same FP32-rounded inputs; the device
    keeps each iterate in FP32, the oracle in FP64), gradients of the first
    against differences of the oracle (per-component metric of
    tests/test_gpu_gradients.py)."""
    import paper_2512_13319_amd as ms
    from tests.test_gpu_gradients import GTOL, grad_err
    wl = workloads.config(5).rounded(dtype)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype])
    r = ms.iterated_nonlinear(p, wl.n_iter, covariances=True, loglik=True, objective=True,
                              grad=True)
    torch.cuda.synchronize()
    segs = np.array([0, 101, 255])
    sub, rows = sub_workload(wl, segs)
    o = cref.iterate(sub)
    e_xs = rel_err(r["xs"].cpu().numpy().T[rows], o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"][:, torch.as_tensor(rows, device=r["Ps"].device)], 3),
                   o["Ps"])
    print(f"cfg5 {dtype}: xs {e_xs:.2e} Ps {e_Ps:.2e}")
    assert e_xs <= TOL[dtype] and e_Ps <= TOL[dtype]
    # gradients on the last linear problem (linearisation point frozen) by a
    # five-point central-difference stencil of the oracle, for the first
    # sampled segment.  The log-likelihood is ~2e5 in magnitude, so a plain
    # two-point difference with a tiny step loses ~1e-5 to cancellation; the
    # fourth-order stencil at h = 3e-3 |theta_i| is accurate to ~1e-8.
    one, _ = sub_workload(wl, segs[:1])
    xbar = o["xbar"][:, : one.n_states]
    gl = r["g_loglik"].cpu().numpy()[segs[0]]
    gm = r["g_obj"].cpu().numpy()[segs[0]]
    th = one.theta[0].copy()
    fd = np.zeros((2, th.size))
    for i in range(th.size):
        h = 3e-3 * abs(th[i])
        vals = {}
        for k in (-2, -1, 1, 2):
            w = workloads.Workload(**{**one.__dict__})
            w.theta = one.theta.copy()
            w.theta[0, i] = th[i] + k * h
            oo = cref.smooth(w, xbar)
            vals[k] = (oo["loglik"][0], oo["mstar"][0])
        fd[:, i] = [(-vals[2][j] + 8 * vals[1][j] - 8 * vals[-1][j] + vals[-2][j]) / (12 * h)
                    for j in (0, 1)]
        print(f"cfg5 {dtype} theta[{i}]: dl {gl[i]:.10e} fd {fd[0, i]:.10e}  "
              f"dM {gm[i]:.10e} fd {fd[1, i]:.10e}")
    el, em = grad_err(gl, fd[0], dtype), grad_err(gm, fd[1], dtype)
    print(f"cfg5 {dtype} gradients: loglik {el:.1e} obj {em:.1e}")
    assert el <= GTOL[dtype] and em <= GTOL[dtype]
