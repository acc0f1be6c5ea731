"""Checkpointed adjoint on the GPU: map_smooth_checkpointed keeps only the
filter's block carries, and map_backward rebuilds S, v from them.

The rebuilt planes come from the same kernels, inputs and carries as the
forward pass's, so they must equal them bit for bit, and so must x* and P^s.
The per-segment sums (objective, gradients) are reduced with atomic adds
across blocks, whose order varies, so they are held to 1e-12 of the largest
component instead. Against the oracle the bar is the gradient bar of the
saved-plane adjoint: 1e-6 per component in FP64."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref, ref
from tests.test_gpu_gradients import GTOL, TORCH_DT, _case, _seg_xbar, grad_err

pytestmark = pytest.mark.gpu

SUM_TOL = 1e-12


def _sum_err(a, b):
    a = np.atleast_2d(a.double().cpu().numpy())
    b = np.atleast_2d(b.double().cpu().numpy())
    scale = np.maximum(np.abs(b).max(axis=-1, keepdims=True), 1e-300)
    return float((np.abs(a - b) / scale).max())


def _same_states(p, a, b, key):
    """Bitwise equality over the states (the tiled layout's padding past the
    last state is never written)."""
    comps = {"S": p.nsym, "v": p.nx, "xs": p.nx, "Ps": p.nsym}[key]
    return torch.equal(p.natural(a, comps), p.natural(b, comps))


def _ragged(dtype):
    """About 40k states in 7 ragged segments (one of a single step, one
    shorter than a tile), so that every schedule has several blocks (8192
    states per block at 32 per lane, 1024 at 4) and segment starts fall
    inside blocks, tiles and lanes."""
    wl = workloads.cv_batched(n_seg=7, lens=[9000, 1, 700, 12000, 33, 8000, 10262], seed=91,
                              gamma=0.2)
    return wl.rounded(dtype)


def _problem(wl, dtype, chunk, xbar=None):
    import paper_2512_13319_amd as ms
    return ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk,
                                    xbar=None if xbar is None else torch.tensor(xbar))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("chunk", [4, 8, 16, 32])
def test_checkpointed_forward_and_backward(chunk, dtype):
    import paper_2512_13319_amd as ms
    wl = _ragged(dtype)
    p = _problem(wl, dtype, chunk)
    print(f"ragged cv {dtype} chunk {chunk}: {wl.n_states} states", flush=True)
    r0 = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False)
    r1 = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False,
                   checkpoint=True)
    torch.cuda.synchronize()
    assert r1["ckpt"].numel() == ms.checkpoint_bytes(p)
    # the checkpointed forward pass is map_smooth on the same schedule
    for k in ("S", "v", "xs", "Ps"):
        assert _same_states(p, r0[k], r1[k], k), k
    for k in ("loglik", "obj", "g_loglik", "g_obj"):
        assert _sum_err(r1[k], r0[k]) <= SUM_TOL, k
    rng = np.random.default_rng(92)
    w = torch.tensor(rng.normal(size=(wl.nx, wl.n_states)))
    b0 = ms.backward(p, r1["S"], r1["v"], covariances=True, objective=True, natural=False,
                     g_xs=w, elem_grads=dtype == "f64")
    b1 = ms.backward(p, None, None, covariances=True, objective=True, natural=False, g_xs=w,
                     elem_grads=dtype == "f64", ckpt=r1["ckpt"])
    torch.cuda.synchronize()
    # rebuilt filter planes, trajectory and covariances: bit for bit
    for k in ("S", "v", "xs", "Ps"):
        assert _same_states(p, b1[k], r1[k], k), k
    # sums: as the fused forward pass; and as the adjoint from saved planes,
    # whose trajectory maps are built from the stored planes (the same values
    # in FP64, rounded ones with FP32 storage: there the FP32 bar of the
    # saved-plane adjoint against the fused pass applies)
    tol = 1e-10 if dtype == "f64" else 1e-4
    for k in ("obj", "g_loglik", "g_obj"):
        e1, e0 = _sum_err(b1[k], r1[k]), _sum_err(b1[k], b0[k])
        print(f"  {k}: vs forward {e1:.1e}, vs saved planes {e0:.1e}")
        assert e1 <= SUM_TOL and e0 <= tol, k
    e = _sum_err(b1["g_xs_theta"], b0["g_xs_theta"])
    e_mu = _sum_err(p.natural(b1["mu"], p.nx), p.natural(b0["mu"], p.nx))
    print(f"  g_xs_theta vs saved planes {e:.1e}, mu {e_mu:.1e}")
    assert e <= tol and e_mu <= tol
    if dtype == "f64":
        n = 2 * ms.elem_grad_size(p)
        ge1 = ms.from_tiled(b1["g_elems"], n, wl.n_states)
        ge0 = ms.from_tiled(b0["g_elems"], n, wl.n_states)
        scale = ge0.abs().amax(dim=1, keepdim=True).clamp_min(1e-300)
        e = float(((ge1 - ge0).abs() / scale).max())
        print(f"  g_elems vs saved planes {e:.1e}")
        assert e <= 1e-10


def _oracle_case(model):
    """Workloads of 1400-2900 states: two or three blocks at 4 states per
    lane (1024 states per block), segment starts inside blocks."""
    if model == "cv":
        wl = workloads.cv_batched(n_seg=4, lens=[900, 5, 1300, 640], seed=95, gamma=0.25)
    elif model == "vdp":
        wl = workloads.vdp(T=1500, dt=0.01, seed=96, n_iter=3)
    elif model == "lorenz63":
        wl = workloads.lorenz63(n_seg=2, T=800, dt=0.005, seed=97, n_iter=2)
    else:
        wl = workloads.ct(n_seg=2, T=700, seed=98, n_iter=2)
    wl = wl.rounded("f64")
    xbar = None if model == "cv" else cref.iterate(wl)["xbar"]
    return wl, xbar


@pytest.mark.parametrize("model", ["cv", "vdp", "lorenz63", "ct"])
def test_checkpointed_gradients_match_oracle(model):
    """Fisher and envelope gradients and the trajectory VJP from the
    checkpointed adjoint (4 states per lane) against autograd of the
    sequential oracle (linearisation point fixed), every segment, FP64."""
    import paper_2512_13319_amd as ms
    chunk = 4
    wl, xbar = _oracle_case(model)
    p = _problem(wl, "f64", chunk, xbar)
    rng = np.random.default_rng(93)
    w = rng.normal(size=(wl.nx, wl.n_states))
    r = ms.smooth(p, covariances=False, loglik=False, objective=False, natural=False,
                  checkpoint=True)
    b = ms.backward(p, None, None, covariances=False, objective=False, natural=False,
                    g_xs=torch.tensor(w), ckpt=r["ckpt"])
    torch.cuda.synchronize()
    for s in range(wl.n_seg):
        seg = ref.workload_segment(wl, s)
        st = wl.seg_states(s)
        xb = _seg_xbar(wl, xbar, s)
        gl, gm, _ = ref.gradients(wl.model, wl.nx, seg, xb)
        gx = ref.trajectory_vjp(wl.model, wl.nx, seg, xb, torch.tensor(w[:, st].T.copy()))
        errs = [grad_err(b["g_loglik"][s].cpu().numpy(), gl.numpy()),
                grad_err(b["g_obj"][s].cpu().numpy(), gm.numpy()),
                grad_err(b["g_xs_theta"][s].cpu().numpy(), gx.numpy())]
        print(f"{model} chunk {chunk} segment {s}: loglik {errs[0]:.1e} obj {errs[1]:.1e} "
              f"vjp {errs[2]:.1e}")
        assert max(errs) <= GTOL["f64"], (s, errs)


def test_mapsmooth_checkpointed_autograd():
    """MapSmooth with checkpoint=True: the same gradient as without it (which
    the oracle pins in the MapSmooth autograd test), from a cotangent on the
    log-likelihood, the objective and x*."""
    import paper_2512_13319_amd as ms
    wl, _, p = _case("cv")
    rng = np.random.default_rng(94)
    w = torch.tensor(rng.normal(size=(wl.nx, wl.n_states)), device="cuda")
    grads = []
    for ck in (False, True):
        theta = torch.tensor(wl.theta, dtype=torch.float64, device="cuda").requires_grad_(True)
        xs, ll, obj = ms.MapSmooth.apply(theta, p, ck)
        loss = 0.7 * ll.sum() - 1.3 * obj.sum() + (xs * w).sum()
        g, = torch.autograd.grad(loss, theta)
        grads.append(g)
    e = _sum_err(grads[1], grads[0])
    print(f"MapSmooth checkpointed vs saved planes: {e:.1e}")
    assert e <= SUM_TOL


@pytest.mark.parametrize("cfg,dtype", [(2, "f64"), (4, "f32")])
def test_checkpointed_adjoint_full_size(cfg, dtype):
    """The timed workloads in full (one 2^20-step trajectory in FP64; 4096
    ragged segments, 1.6e7 steps, FP32 storage) on the library's flat
    schedule: the checkpoint is below 0.1 % of the S, v planes (14 KB and
    222 KB), the rebuilt planes and x* equal the forward pass's bit for bit,
    and the gradients equal the forward pass's."""
    import paper_2512_13319_amd as ms
    wl = workloads.config(cfg).rounded(dtype)
    p = _problem(wl, dtype, 0)
    print(f"cfg{cfg} {dtype}: {wl.n_states} states", flush=True)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False,
                  checkpoint=True)
    nbytes = r["ckpt"].numel()
    assert nbytes <= wl.n_states * 14 * 8 // 1000    # below 0.1 % of the FP64 S, v planes
    S, v, xs = r["S"].clone(), r["v"].clone(), r["xs"].clone()
    r["S"].fill_(float("nan"))
    r["v"].fill_(float("nan"))
    b = ms.backward(p, r["S"], r["v"], covariances=True, objective=True, natural=False,
                    ckpt=r["ckpt"])
    torch.cuda.synchronize()
    for k, ref_k in (("S", S), ("v", v), ("xs", xs), ("Ps", r["Ps"])):
        assert _same_states(p, b[k], ref_k, k), k
    for k in ("obj", "g_loglik", "g_obj"):
        e = _sum_err(b[k], r[k])
        print(f"  {k}: {e:.1e}")
        assert e <= SUM_TOL, k


@pytest.mark.parametrize("case", ["empty_segments", "no_steps", "f32_arithmetic"])
def test_checkpointed_edge_cases(case):
    """Empty segments between others, a problem without steps (every
    segment its prior, one block), and FP32 arithmetic (an FP32 checkpoint):
    the rebuilt planes, x* and P^s equal the forward call's bit for bit."""
    import paper_2512_13319_amd as ms
    arith, dtype, chunk = "f64", "f64", 4
    if case == "empty_segments":
        wl = workloads.cv_batched(lens=[0, 1500, 0, 0, 533, 0, 1, 0], seed=18)
    elif case == "no_steps":
        wl = workloads.cv_batched(lens=[0, 0, 0, 0, 0], seed=20)
    else:
        wl, arith, dtype, chunk = _ragged("f32"), "f32", "f32", 16
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk, arith=arith)
    print(f"{case}: {wl.n_states} states", flush=True)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False,
                  checkpoint=True)
    b = ms.backward(p, None, None, covariances=True, objective=True, natural=False,
                    ckpt=r["ckpt"])
    torch.cuda.synchronize()
    # 14 values of the arithmetic type per block
    assert r["ckpt"].numel() == ms.checkpoint_bytes(p)
    assert r["ckpt"].numel() % (14 * (4 if arith == "f32" else 8)) == 0
    for k in ("S", "v", "xs", "Ps"):
        assert _same_states(p, b[k], r[k], k), k
    for k in ("obj", "g_loglik", "g_obj"):
        e = _sum_err(b[k], r[k])
        print(f"  {k}: {e:.1e}")
        assert e <= SUM_TOL, k
