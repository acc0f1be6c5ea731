"""GPU parity of the exact (Van Loan) discretisation of time-invariant linear
models: the library's host-side terms (map_lti_exact_terms) run through the
general linear model's kernels, against the oracle's filter and smoother on
the oracle's own exact terms (scipy expm).  Tolerances as in test_gpu_parity."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref, lti
from tests.test_gpu_parity import TOL, TORCH_DT, planes_T, rel_err, sym_full

pytestmark = pytest.mark.gpu


def rel_err_floor(gpu, refv):
    """rel_err with each component's scale floored at 1e-6 of the largest
    one: the square root of C / dt is not unique, and where the oracle's
    (LAPACK eigh) mixes the two identical axes, structurally zero cross-axis
    covariances come out as rounding noise (~1e-20 of the largest entry) on its
    side and as exact zeros on the library's side (its Jacobi rotations skip
    zero entries).  Only such components reach the floor."""
    g = np.asarray(gpu, dtype=np.float64).reshape(gpu.shape[0], -1)
    r = np.asarray(refv, dtype=np.float64).reshape(refv.shape[0], -1)
    den = np.maximum(np.abs(r).max(0), 1e-6 * np.abs(r).max())
    return float((np.abs(g - r).max(0) / den).max())


def _cv_terms(gamma, q, r, c):
    F = np.zeros((4, 4)); F[:2, 2:] = np.eye(2); F[2:, 2:] = -gamma * np.eye(2)
    L = np.vstack([np.zeros((2, 2)), np.eye(2)])
    return F, np.asarray(c, dtype=np.float64), L, q * np.eye(2), np.hstack([np.eye(2), np.zeros((2, 2))]), \
        np.array([0.02, -0.03]), r * np.eye(2)


def exact_pair(T, dt, gamma, q=0.5, r=0.05, c=(0, 0, 0.15, -0.1), seed=61, dtype="f64"):
    """(GPU workload with the library's terms, shared; oracle workload with the
    oracle's terms, per step) for one constant-velocity track."""
    import paper_2512_13319_amd as ms
    base = workloads.cv(T=T, d=2, dt=dt, gamma=gamma, q=q, r=r, m0=[5, 5, 0, 0],
                        P0=1e-2 * np.eye(4), seed=seed).rounded(dtype)
    F, c, L, W, H, rr, R = _cv_terms(gamma, q, r, c)
    gl = ms.lti_exact_terms(F, c, L, W, dt)
    ol = lti.implicit_equivalent(F, c, L, W, dt)
    mk = lambda lin: workloads.Workload(name="lti_exact", model="linear", nx=4, ny=2, nw=4,
                                        seg_off=base.seg_off, dt=base.dt, y=base.y,
                                        theta=np.zeros((1, 0)), m0=base.m0, P0=base.P0,
                                        x_true=base.x_true, lin=lin, dtype=dtype)
    per = lambda m: np.broadcast_to(m, (T,) + m.shape)
    wg = mk(dict(F=gl[0], c=gl[1], L=gl[2], W=gl[3], H=H, r=rr, R=R))
    wo = mk(dict(F=per(ol[0]), c=per(ol[1]), L=ol[2], W=ol[3], H=per(H), r=per(rr), R=R))
    return wg, wo


@pytest.mark.parametrize("shared_dt", [False, True])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("T,gamma", [(3 * 1024 + 77, 0.0), (2055, 0.6)])
def test_lti_exact_parity(T, gamma, dtype, shared_dt):
    """shared_dt: one step length for all steps, so that every term of the
    general linear model is shared (the kernels then build a step's terms once
    per block); otherwise the same value given per step."""
    import dataclasses

    import paper_2512_13319_amd as ms
    wg, wo = exact_pair(T, 1e-3, gamma, dtype=dtype)
    if shared_dt:
        wg = dataclasses.replace(wg, dt=np.asarray(float(wg.dt[0])))
    if dtype == "f32":
        # the FP32 run stores rounded terms; the oracle sees the same rounding
        for k in ("F", "c", "L", "W", "H", "r", "R"):
            wo.lin[k] = np.asarray(wo.lin[k], dtype=np.float32).astype(np.float64)
            wg.lin[k] = np.asarray(wg.lin[k], dtype=np.float32).astype(np.float64)
    o = cref.smooth(wo)
    p = ms.problem_from_workload(wg, dtype=TORCH_DT[dtype])
    r = ms.smooth(p, covariances=True, loglik=True, objective=True)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err_floor(sym_full(ms, r["Ps"], 4), o["Ps"])
    e_ll = abs(r["loglik"].item() - o["loglik"][0]) / abs(o["loglik"][0])
    e_ob = abs(r["obj"].item() - o["mstar"][0]) / abs(o["mstar"][0])
    msg = f"lti exact T={T} gamma={gamma} {dtype}: xs {e_xs:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e} obj {e_ob:.2e}"
    print(msg)
    tol = TOL[dtype]
    assert max(e_xs, e_Ps, e_ll, e_ob) <= tol, msg


def test_lti_exact_full_wiener_velocity():
    """The benchmark's 2^20-step Wiener-velocity track with exact dynamics."""
    import paper_2512_13319_amd as ms
    wg, wo = exact_pair(2 ** 20, 1e-3, 0.0, c=(0, 0, 0, 0), seed=2)
    o = cref.smooth(wo)
    p = ms.problem_from_workload(wg, dtype=torch.float64)
    r = ms.smooth(p, covariances=True, loglik=True, objective=False)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err_floor(sym_full(ms, r["Ps"], 4), o["Ps"])
    e_ll = abs(r["loglik"].item() - o["loglik"][0]) / abs(o["loglik"][0])
    print(f"lti exact full: xs {e_xs:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e}")
    assert max(e_xs, e_Ps, e_ll) <= 1e-9
