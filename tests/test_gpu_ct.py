"""GPU parity of the coordinated-turn model (Sec. 5.2): iterated linearisation
(5 Gauss--Newton iterations from m0) through the C-ABI against the C oracle,
FP64 and FP32 storage, every schedule, the two-filter form, gradients against
autograd of the torch oracle and differences of the C oracle, the bearing wrap, and the 64 x 2^14-step
workload that the benchmark times (sampled segments).  Tolerances as in
test_gpu_parity (1e-9 FP64, 1e-4 FP32, gradients 1e-6)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref
from tests.test_gpu_parity import TOL, TORCH_DT, planes_T, rel_err, sym_full
from tests.test_gpu_fullsize import state_rows, sub_workload

pytestmark = pytest.mark.gpu

CASES = {
    # 3 x 901 states: two full tiles and a ragged third
    "ct_three": lambda: workloads.ct(n_seg=3, T=900, seed=91),
    # 2056 states: the final 8-state tile runs on the last lane of the tile before it
    "ct_merged_tail": lambda: workloads.ct(n_seg=1, T=2055, seed=92),
}


def _run(wl, dtype, chunk=0, grad=False):
    import paper_2512_13319_amd as ms
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk)
    r = ms.iterated_nonlinear(p, wl.n_iter, covariances=True, loglik=True, objective=True,
                              grad=grad)
    torch.cuda.synchronize()
    return ms, r


def _compare(ms, wl, r, o, tol, tag):
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_xb = rel_err(planes_T(r["xbar"]), o["xbar"].T)
    e_Ps = rel_err(sym_full(ms, r["Ps"], 5), o["Ps"])
    e_ll = np.abs(r["loglik"].cpu().numpy() - o["loglik"]).max() / np.abs(o["loglik"]).max()
    e_ob = np.abs(r["obj"].cpu().numpy() - o["mstar"]).max() / np.abs(o["mstar"]).max()
    msg = f"{tag}: xs {e_xs:.2e} xbar {e_xb:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e} obj {e_ob:.2e}"
    print(msg)
    assert max(e_xs, e_xb, e_Ps, e_ll, e_ob) <= tol, msg


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_ct_iterated_parity(case, dtype):
    wl = CASES[case]().rounded(dtype)
    o = cref.iterate(wl)
    ms, r = _run(wl, dtype)
    _compare(ms, wl, r, o, TOL[dtype], f"ct {case} {dtype}")


@pytest.mark.parametrize("chunk", [8, 16, 32])
def test_ct_iterated_parity_schedules(chunk):
    wl = CASES["ct_three"]()
    o = cref.iterate(wl)
    ms, r = _run(wl, "f64", chunk)
    _compare(ms, wl, r, o, 1e-9, f"ct ct_three f64 chunk {chunk}")


def test_ct_two_filter_parity():
    """The two-filter form on the coordinated-turn model, linearised about the
    simulated path."""
    import paper_2512_13319_amd as ms
    wl = CASES["ct_three"]()
    xb = np.ascontiguousarray(wl.x_true)
    o = cref.two_filter(wl, xb)
    p = ms.problem_from_workload(wl, dtype=torch.float64, xbar=torch.as_tensor(xb))
    r = ms.two_filter_smooth(p, covariances=True, loglik=False)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"], 5), o["Ps"])
    print(f"ct two-filter: xs {e_xs:.2e} Ps {e_Ps:.2e}")
    assert e_xs <= 1e-9 and e_Ps <= 1e-9


def test_ct_bearing_branch_does_not_matter():
    """Bearings given on another branch (shifted by +-2 pi) give the same
    iterates, likelihood and objective."""
    wl = CASES["ct_three"]()
    w2 = workloads.Workload(**{**wl.__dict__})
    w2.y = wl.y.copy()
    k = np.arange(0, w2.y.shape[1], 5)
    w2.y[1, k] += 2 * np.pi * np.where(k % 2 == 0, 1.0, -1.0)
    ms, a = _run(wl, "f64")
    _, b = _run(w2, "f64")
    for key in ("xs", "Ps"):
        e = rel_err(planes_T(b[key]), planes_T(a[key]))
        assert e <= 1e-12, (key, e)
    assert np.abs(a["loglik"].cpu().numpy() - b["loglik"].cpu().numpy()).max() <= \
        1e-12 * np.abs(a["loglik"].cpu().numpy()).max()


def test_ct_gradients_against_autograd_and_differences():
    """d loglik / d theta (Fisher identity) and d M* / d theta (envelope) of
    the last linear problem, theta = (sv, sw, r1, r2), with the linearisation
    point fixed: against autograd of the torch oracle at 1e-6, and against
    five-point differences of the C oracle at 1e-4.  The differences need a
    step per parameter: sv, sw (5e-4, 0.02) enter through their squares and
    move a log-likelihood of ~5e3 by ~1e-2 per unit, so a step of 1e-3 |theta|
    is roundoff-bound; 0.1 |theta| is used there and 3e-3 |theta| for r1, r2."""
    from oracle import ref
    from tests.test_gpu_gradients import grad_err
    wl = workloads.ct(n_seg=2, T=1500, seed=93)
    o = cref.iterate(wl)
    ms, r = _run(wl, "f64", grad=True)
    gl = r["g_loglik"].cpu().numpy()
    gm = r["g_obj"].cpu().numpy()
    xbar = o["xbar"]
    steps = (0.1, 0.1, 3e-3, 3e-3)
    for s in range(2):
        one, rows = sub_workload(wl, np.array([s]))
        xb = np.ascontiguousarray(xbar[:, rows])
        al, am, _ = ref.gradients("ct", 5, ref.workload_segment(one, 0), torch.tensor(xb.T))
        al, am = al.numpy(), am.numpy()
        # per component (metric of tests/test_gpu_gradients.py)
        assert grad_err(gl[s], al) <= 1e-6 and grad_err(gm[s], am) <= 1e-6, (gl[s], al, gm[s], am)
        th = one.theta[0].copy()
        for i in range(4):
            h = steps[i] * abs(th[i])
            vals = {}
            for k in (-2, -1, 1, 2):
                w = workloads.Workload(**{**one.__dict__})
                w.theta = one.theta.copy()
                w.theta[0, i] = th[i] + k * h
                oo = cref.smooth(w, xb)
                vals[k] = (oo["loglik"][0], oo["mstar"][0])
            fd_l, fd_m = ((-vals[2][j] + 8 * vals[1][j] - 8 * vals[-1][j] + vals[-2][j]) / (12 * h)
                          for j in (0, 1))
            print(f"ct seg {s} theta[{i}]: dl {gl[s, i]:.10e} autograd {al[i]:.10e} fd {fd_l:.6e}"
                  f"  dM {gm[s, i]:.10e} autograd {am[i]:.10e} fd {fd_m:.6e}")
            assert abs(gl[s, i] - fd_l) <= 1e-4 * abs(fd_l)
            assert abs(gm[s, i] - fd_m) <= 1e-4 * abs(fd_m)


def test_ct_full_workload_sampled():
    """64 tracks of 2^14 steps, 5 iterations (the benchmark's coordinated-turn
    workload), FP64; the oracle recomputes a sample of tracks."""
    wl = workloads.ct()
    ms, r = _run(wl, "f64")
    segs = np.array([0, 17, 63])
    sub, rows = sub_workload(wl, segs)
    o = cref.iterate(sub)
    e_xs = rel_err(planes_T(r["xs"])[rows], o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"][:, torch.as_tensor(rows, device=r["Ps"].device)], 5),
                   o["Ps"])
    ll = r["loglik"].cpu().numpy()[segs]
    e_ll = np.abs(ll - o["loglik"]).max() / np.abs(o["loglik"]).max()
    print(f"ct full (3 sampled tracks): xs {e_xs:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e}")
    assert e_xs <= 1e-9 and e_Ps <= 1e-9 and e_ll <= 1e-9
