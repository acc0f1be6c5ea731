"""Sub-stepped blocks on the GPU (n_sub Euler substeps of the element ODE per
grid step, the paper's T blocks x n substeps) and their dense output, against
the block oracle (`oracle/blocks.py`: conditioning on the blocks' backward
transitions in covariance form, pinned to the Kalman filter / RTS smoother
at one substep and to the fine-grid smoother as the substep shrinks).
Metric as test_gpu_parity: 1e-9 FP64, 1e-4 FP32, each component relative to
its own scale; the FP32 run and the FP64 oracle see the same FP32-rounded
inputs."""
import numpy as np
import pytest
import torch

import workloads
from oracle import blocks as oracle_blocks
from tests.test_gpu_parity import TOL, TORCH_DT, planes_T, rel_err, sym_full

pytestmark = pytest.mark.gpu


def _cv_blocks(n_sub, dtype):
    wl = workloads.cv_batched(lens=[n_sub * k for k in (230, 1, 47, 3, 120)], seed=95,
                              gamma=0.2)
    return workloads.blocks(wl, n_sub).rounded(dtype)


def _check(ms, p, wl, o, dtype, tag):
    r = ms.smooth(p, covariances=True, loglik=False, objective=False, natural=False)
    d = ms.dense_output(p, r["S"], r["v"], r["xs"])
    torch.cuda.synchronize()
    nx, n = wl.nx, wl.n_sub
    nat = lambda k, c: p.natural(r[k], c)
    e = {"xs": rel_err(planes_T(nat("xs", nx)), o["xs"]),
         "Ps": rel_err(sym_full(ms, nat("Ps", p.nsym), nx), o["Ps"]),
         "S": rel_err(sym_full(ms, nat("S", p.nsym), nx), o["S"])}
    vref = o["v"] if dtype == "f64" else o["m"]
    e["v"] = rel_err(planes_T(nat("v", nx)), vref)
    # dense output at the interior substeps of every block (not at segment starts)
    heads = wl.seg_off[:-1] + np.arange(wl.n_seg)
    rows = np.setdiff1d(np.arange(wl.n_states), heads)
    xd = d["xd"].double().cpu().numpy()          # [n-1, nx, n_states]
    e["dense_xs"] = rel_err(xd[:, :, rows].transpose(2, 0, 1).reshape(len(rows), -1),
                            o["dense_xs"][rows].reshape(len(rows), -1))
    Sd = d["Sd"]                                  # [n-1, nsym, n_states]
    Sfull = np.stack([sym_full(ms, Sd[j][:, torch.as_tensor(rows, device=Sd.device)], nx)
                      for j in range(n - 1)], 1)
    e["dense_S"] = rel_err(Sfull.reshape(len(rows), -1), o["dense_S"][rows].reshape(len(rows), -1))
    vd = d["vd"].double().cpu().numpy()[:, :, rows].transpose(2, 0, 1)
    vdref = (o["dense_v"] if dtype == "f64" else o["dense_m"])[rows]
    e["dense_v"] = rel_err(vd.reshape(len(rows), -1), vdref.reshape(len(rows), -1))
    msg = "%s %s: " % (tag, dtype) + " ".join("%s %.1e" % kv for kv in e.items())
    print(msg)
    assert max(e.values()) <= TOL[dtype], msg


@pytest.mark.parametrize("chunk", [0, 16, 32, -1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cv_blocks_of_ten_substeps(dtype, chunk):
    """Constant velocity (nx = 4), blocks of 10 substeps as in the paper's
    linear experiment, ragged segments (one of a single block), every
    schedule."""
    import paper_2512_13319_amd as ms
    wl = _cv_blocks(10, dtype)
    o = oracle_blocks.smooth(wl)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk)
    _check(ms, p, wl, o, dtype, "cv n_sub 10 chunk %d" % chunk)


def test_block_elements_match_the_oracle():
    """map_build_elements with blocks: the Euler-integrated element of every
    block (A, b, C, eta, J) against the oracle's."""
    import paper_2512_13319_amd as ms
    wl = _cv_blocks(7, "f64")
    p = ms.problem_from_workload(wl, dtype=torch.float64)
    el = ms.build_elements(p).double().cpu().numpy()  # [comps, n_states]
    nx = 4
    from oracle import models
    for s in range(wl.n_seg):
        st = wl.seg_steps(s)
        F, c, L, W, H, r, R = models.terms_numpy("cv", wl.theta[s], np.zeros((1, nx)), nx)
        for k in range(st.start, st.stop):
            h = wl.dt[k] / wl.n_sub
            ys = wl.y[:, k].reshape(wl.n_sub, wl.ny)
            A, b, C, eta, J = oracle_blocks.euler_block(F[0], c[0], L @ W @ L.T, H[0],
                                                        np.linalg.inv(R), r[0], ys, h)[-1]
            i = k + s + 1
            g = el[:, i]
            gA = g[:16].reshape(4, 4)
            gb = g[16:20]
            sym = lambda a: np.array([a[r_][q] for r_ in range(4) for q in range(r_ + 1)])
            gC, geta, gJ = g[20:30], g[30:34], g[34:44]
            for got, ref_ in ((gA, A), (gb, b), (gC, sym(C)), (geta, eta), (gJ, sym(J))):
                assert np.abs(got - ref_).max() <= 1e-11 * max(np.abs(ref_).max(), 1e-300)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vdp_blocks_iterated(dtype):
    """Van der Pol with blocks of 5 substeps, 3 Gauss-Newton iterations (the
    terms of each block linearised at its last state): final iterate, its
    linearisation point and the dense output."""
    import paper_2512_13319_amd as ms
    wl = workloads.blocks(workloads.vdp(T=5 * 400, dt=0.004, seed=96, n_iter=3), 5).rounded(dtype)
    o = oracle_blocks.iterate(wl)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype])
    r = ms.iterated_nonlinear(p, wl.n_iter, covariances=True, loglik=False, objective=False,
                              natural=False)
    torch.cuda.synchronize()
    e_xs = rel_err(planes_T(p.natural(r["xs"], 2)), o["xs"])
    e_xb = rel_err(planes_T(p.natural(r["xbar"], 2)), o["xbar"].T)
    e_Ps = rel_err(sym_full(ms, p.natural(r["Ps"], 3), 2), o["Ps"])
    # dense output of the last linear problem (linearised about r["xbar"])
    p.set_xbar(p.natural(r["xbar"], 2))
    d = ms.dense_output(p, r["S"], r["v"], r["xs"])
    torch.cuda.synchronize()
    xd = d["xd"].double().cpu().numpy()[:, :, 1:].transpose(2, 0, 1)
    e_d = rel_err(xd.reshape(xd.shape[0], -1), o["dense_xs"][1:].reshape(xd.shape[0], -1))
    msg = f"vdp blocks {dtype}: xs {e_xs:.1e} xbar {e_xb:.1e} Ps {e_Ps:.1e} dense {e_d:.1e}"
    print(msg)
    assert max(e_xs, e_xb, e_Ps, e_d) <= TOL[dtype], msg
