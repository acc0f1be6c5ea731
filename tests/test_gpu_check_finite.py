"""MAP_CHECK_FINITE through the C-ABI: with the flag, a call whose results hold
a non-finite value (here from one NaN measurement) returns MAP_E_NUMERIC after
its stream work; the status lives in the workspace and is cleared, so the next
clean call passes.  A clean problem gives the same results with and without
the check, and without the flag nothing is checked."""
import numpy as np
import pytest
import torch

import workloads
from paper_2512_13319_amd import _lib

pytestmark = pytest.mark.gpu

MAP_E_NUMERIC = -5


def _ms():
    import paper_2512_13319_amd as ms
    return ms


def _cv(seed=41):
    return workloads.cv_batched(n_seg=7, lmin=6.0, lmax=11.0, seed=seed)


def _with_nan(wl, k):
    y = wl.y.copy()
    y[0, k] = np.nan
    bad = workloads.Workload(**{**wl.__dict__})
    bad.y = y
    return bad


def test_clean_problem_same_results_with_and_without_the_check():
    ms = _ms()
    wl = _cv()
    r0 = ms.smooth(ms.problem_from_workload(wl), covariances=True, loglik=True, objective=True,
                   grad=True)
    r1 = ms.smooth(ms.problem_from_workload(wl, check_finite=True), covariances=True,
                   loglik=True, objective=True, grad=True)
    torch.cuda.synchronize()
    # per-state outputs are deterministic; per-segment sums are added with
    # atomics in whatever order the blocks finish
    for k in ("xs", "Ps"):
        a, b = r0[k].double().cpu().numpy(), r1[k].double().cpu().numpy()
        assert np.array_equal(a, b), k
    for k in ("loglik", "obj", "g_loglik", "g_obj"):
        a, b = r0[k].double().cpu().numpy(), r1[k].double().cpu().numpy()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), k


@pytest.mark.parametrize("form", ["smooth", "filter", "two_filter"])
def test_nan_measurement_is_reported_then_cleared(form):
    ms = _ms()
    wl = _cv()
    k = int(wl.seg_off[3]) + 5  # a step inside the fourth segment
    p = ms.problem_from_workload(_with_nan(wl, k), check_finite=True)
    run = {"smooth": lambda q: ms.smooth(q, covariances=True, loglik=True, objective=True),
           "filter": lambda q: ms.filter_scan(q, moments=True, loglik=True),
           "two_filter": lambda q: ms.two_filter_smooth(q, covariances=True, loglik=True)}[form]
    print(f"check_finite {form}: NaN at step {k}", flush=True)
    with pytest.raises(_lib.MapError) as ei:
        run(p)
    assert ei.value.status == MAP_E_NUMERIC and "non-finite" in str(ei.value)
    # same problem object (same workspace), measurement repaired in place
    p.y.copy_(ms.problem_from_workload(wl).y)
    r = run(p)
    torch.cuda.synchronize()
    assert all(torch.isfinite(v).all() for v in r.values() if torch.is_tensor(v))


def test_without_the_flag_nothing_is_checked():
    ms = _ms()
    wl = _cv()
    p = ms.problem_from_workload(_with_nan(wl, int(wl.seg_off[2]) + 3))
    r = ms.smooth(p, covariances=True, loglik=True, objective=True)
    torch.cuda.synchronize()
    assert not torch.isfinite(r["xs"]).all()


def test_iterated_nonlinear_reports():
    ms = _ms()
    wl = workloads.ct(n_seg=4, T=512, seed=43)
    p = ms.problem_from_workload(_with_nan(wl, 700), check_finite=True)
    with pytest.raises(_lib.MapError) as ei:
        ms.iterated_nonlinear(p, 3, covariances=True, loglik=True, objective=True)
    assert ei.value.status == MAP_E_NUMERIC
