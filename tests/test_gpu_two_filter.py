"""GPU parity of the two-filter smoother (Sec. 4.3, eq. twofilter) through the
C-ABI against the oracle's two-filter smoother, on the cases of the RTS parity
tests (tails, merged final tiles, segment starts inside tiles, singular Q,
general time-varying models), two nonlinear models linearised about a fixed
path, every schedule, and the full 2^20-step constant-velocity workload.
Metric and tolerances as in test_gpu_parity (1e-9 FP64, 1e-4 FP32)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref
from tests.test_gpu_parity import CASES, TOL, TORCH_DT, planes_T, rel_err, sym_full

pytestmark = pytest.mark.gpu

NONLINEAR = {
    "vdp_fixed_xbar": lambda: workloads.vdp(T=3000, seed=31),
    "lorenz_fixed_xbar": lambda: workloads.lorenz63(n_seg=5, T=700, seed=32),
}
ALL = {**CASES, **NONLINEAR}


def _xbar(wl, dtype):
    if wl.model not in ("vdp", "lorenz63"):
        return None
    xb = wl.x_true.astype(np.float32).astype(np.float64) if dtype == "f32" else wl.x_true
    return np.ascontiguousarray(xb)


def _check(case, dtype, chunk):
    import paper_2512_13319_amd as ms
    wl = ALL[case]().rounded(dtype)
    xb = _xbar(wl, dtype)
    o = cref.two_filter(wl, xb)
    ll_ref = cref.smooth(wl, xb)["loglik"]
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk,
                                 xbar=None if xb is None else torch.as_tensor(xb))
    r = ms.two_filter_smooth(p, covariances=True, loglik=True)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"], wl.nx), o["Ps"])
    ll = r["loglik"].cpu().numpy()
    e_ll = np.abs(ll - ll_ref).max() / np.abs(ll_ref).max()
    msg = f"two-filter {case} {dtype} chunk {chunk}: xs {e_xs:.2e} Ps {e_Ps:.2e} ll {e_ll:.2e}"
    print(msg)
    tol = TOL[dtype]
    assert e_xs <= tol and e_Ps <= tol and e_ll <= tol, msg
    return r


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(ALL))
def test_two_filter_parity(case, dtype):
    _check(case, dtype, 0)


@pytest.mark.parametrize("chunk", [8, 16, 32])
@pytest.mark.parametrize("case", ["batched_tail_heads", "cv_tail8_merged", "linear_tv",
                                  "lorenz_fixed_xbar", "batched_many_blocks"])
def test_two_filter_parity_schedules(case, chunk):
    _check(case, "f64", chunk)


def test_two_filter_without_covariances_and_rts_agree():
    """Ps = NULL takes the kernel without the covariance; the means equal the
    RTS form (map_smooth) of the same problem."""
    import paper_2512_13319_amd as ms
    wl = CASES["batched_tail_heads"]()
    p = ms.problem_from_workload(wl, dtype=torch.float64)
    a = ms.two_filter_smooth(p, covariances=False, loglik=False)
    b = ms.smooth(p, covariances=False, loglik=False, objective=False)
    torch.cuda.synchronize()
    assert a["Ps"] is None and a["loglik"] is None
    e = rel_err(planes_T(a["xs"]), planes_T(b["xs"]))
    print(f"two-filter vs RTS means: {e:.2e}")
    assert e <= 1e-9


def test_two_filter_full_cfg2():
    """T = 2^20 constant-velocity workload at the bench's schedule, every state
    against the oracle's two-filter smoother."""
    import paper_2512_13319_amd as ms
    wl = workloads.config(2)
    o = cref.two_filter(wl)
    p = ms.problem_from_workload(wl, dtype=torch.float64)
    r = ms.two_filter_smooth(p, covariances=True, loglik=True)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"], 4), o["Ps"])
    print(f"two-filter cfg2 f64: xs {e_xs:.2e} Ps {e_Ps:.2e}")
    assert e_xs <= 1e-9 and e_Ps <= 1e-9
