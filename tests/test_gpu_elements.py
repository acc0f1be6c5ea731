"""GPU parity of map_build_elements, the element of every state (Sec. 4.2
eq. backwardLQT, one step; Sec. 3.4 for the prior): the prior element
(0, 0, 0, P0^-1 m0, P0^-1) at a segment's first state and the one-step element
(A, b, C, eta, J) of the step ending at every other state.  The reference is
the oracle: on a batch of one-step segments, its run of the steps after a
segment's first state (the two-filter oracle's suffix) is that one step's
element.  Metric: relative max error per component, 1e-12 (FP64)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _ms():
    import paper_2512_13319_amd as ms
    return ms


def _split(e, nx):
    """[n_states, ElemSz] -> A, b, C, eta, J (full matrices)."""
    n = e.shape[0]
    sym = nx * (nx + 1) // 2
    A = e[:, :nx * nx].reshape(n, nx, nx)
    b = e[:, nx * nx: nx * nx + nx]

    def full(block):
        M = np.empty((n, nx, nx))
        c = 0
        for r in range(nx):
            for q in range(r + 1):
                M[:, r, q] = M[:, q, r] = block[:, c]
                c += 1
        return M

    o = nx * nx + nx
    C = full(e[:, o: o + sym])
    eta = e[:, o + sym: o + sym + nx]
    J = full(e[:, o + sym + nx:])
    return dict(A=A, b=b, C=C, eta=eta, J=J)


def _rel(g, r):
    return np.abs(g - r).max() / max(np.abs(r).max(), 1e-300)


CASES = {
    "cv": lambda: workloads.cv_batched(lens=[1] * 40, seed=71),
    "linear_per_step": lambda: workloads.linear_random(T=1, n_seg=40, nx=3, ny=2, nw=3, seed=72),
    "lorenz63": lambda: workloads.lorenz63(n_seg=40, T=1, seed=73),
    "ct": lambda: workloads.ct(n_seg=40, T=1, seed=74),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_elements_match_the_oracle(case):
    ms = _ms()
    wl = CASES[case]()
    nonlinear = wl.model in ("vdp", "lorenz63", "ct")
    xbar = np.ascontiguousarray(wl.x_true) if nonlinear else None
    p = ms.problem_from_workload(wl, xbar=None if xbar is None else torch.as_tensor(xbar))
    e = ms.build_elements(p).double().cpu().numpy().T  # [n_states, ElemSz]
    torch.cuda.synchronize()
    g = _split(e, wl.nx)
    o = cref.two_filter(wl, xbar, suffix=True)["suf"]
    heads = wl.seg_off[:-1] + np.arange(wl.n_seg)   # first state of each segment
    steps = heads + 1                                 # the state its one step ends at
    errs = {k: _rel(g[k][steps], np.asarray(o[k])[heads]) for k in ("A", "b", "C", "eta", "J")}
    # prior elements at the heads
    P0 = np.broadcast_to(wl.P0, (wl.n_seg, wl.nx, wl.nx))
    m0 = np.broadcast_to(wl.m0, (wl.n_seg, wl.nx))
    P0i = np.linalg.inv(P0)
    prior = dict(A=np.zeros_like(P0), b=np.zeros_like(m0), C=np.zeros_like(P0),
                 eta=np.einsum("sij,sj->si", P0i, m0), J=P0i)
    errs.update({"prior " + k: np.abs(g[k][heads] - prior[k]).max() / max(1.0, np.abs(prior[k]).max())
                 for k in prior})
    print(case, {k: "%.1e" % v for k, v in errs.items()})
    assert max(errs.values()) <= TOL, errs
