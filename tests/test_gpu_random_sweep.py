"""Seeded sweep of random ragged batches against the oracle: segment counts and
lengths drawn at random (empty and one-step segments included), every schedule
(4, 8, 16 and the split 32 states per lane, one wavefront per segment), both
storage types, constant-
velocity and general time-varying linear models.  Each case compares x*, P^s,
the log-likelihood and the objective element by element (1e-9 FP64, 1e-4 FP32,
as the other parity tests), each component relative to its own scale."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref
from tests.test_gpu_parity import TOL, TORCH_DT, planes_T, rel_err, sym_full

pytestmark = pytest.mark.gpu


def _lens(rng):
    n_seg = int(rng.integers(1, 40))
    kind = rng.random(n_seg)
    lens = np.where(kind < 0.1, 0, np.where(kind < 0.2, 1,
                    np.floor(2.0 ** rng.uniform(1.0, 12.0, n_seg)).astype(np.int64)))
    if lens.sum() == 0:
        lens[0] = 5
    return lens.astype(np.int64)


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    chunk = int(rng.choice([0, 4, 8, 16, 32, -1]))
    if seed % 3 == 2:
        T = int(rng.integers(50, 3000))
        wl = workloads.linear_random(T=T, nx=3, ny=2, nw=3, n_seg=int(rng.integers(1, 4)),
                                     seed=2000 + seed)
    else:
        wl = workloads.cv_batched(lens=_lens(rng), seed=3000 + seed)
    return wl, chunk


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(12))
def test_random_batches(seed, dtype):
    import paper_2512_13319_amd as ms
    wl, chunk = _case(seed)
    wl = wl.rounded(dtype)
    print(f"sweep seed {seed} {dtype}: model {wl.model}, {wl.n_seg} segments, "
          f"{wl.n_steps} steps, chunk {chunk}", flush=True)
    o = cref.smooth(wl)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk)
    r = ms.smooth(p, covariances=True, loglik=True, objective=True)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    e_xs = rel_err(planes_T(r["xs"]), o["xs"])
    e_Ps = rel_err(sym_full(ms, r["Ps"], wl.nx), o["Ps"])
    ll, ob = r["loglik"].cpu().numpy(), r["obj"].cpu().numpy()
    e_ll = np.abs(ll - o["loglik"]).max() / max(np.abs(o["loglik"]).max(), 1.0)
    e_ob = np.abs(ob - o["mstar"]).max() / max(np.abs(o["mstar"]).max(), 1.0)
    msg = f"seed {seed} {dtype}: xs {e_xs:.1e} Ps {e_Ps:.1e} ll {e_ll:.1e} obj {e_ob:.1e}"
    print(msg)
    assert max(e_xs, e_Ps, e_ll, e_ob) <= tol, msg


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("seed", [s for s in range(12) if s % 3 != 2])
def test_random_batches_checkpointed(seed, dtype):
    """The same random constant-velocity batches through the checkpoint mode
    (map_smooth_checkpointed, then map_backward from the checkpoint, on the
    flat schedule the adjoint resolves): x* against the oracle at the sweep's
    bar, and the rebuilt S, v, x*, P^s equal the forward call's bit for bit."""
    import paper_2512_13319_amd as ms
    wl, chunk = _case(seed)
    wl = wl.rounded(dtype)
    print(f"checkpointed sweep seed {seed} {dtype}: {wl.n_seg} segments, {wl.n_steps} steps, "
          f"chunk {chunk}", flush=True)
    o = cref.smooth(wl)
    p = ms.problem_from_workload(wl, dtype=TORCH_DT[dtype], chunk=chunk)
    f = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=False,
                  checkpoint=True)
    b = ms.backward(p, None, None, covariances=True, objective=True, natural=False,
                    ckpt=f["ckpt"])
    torch.cuda.synchronize()
    comps = dict(S=p.nsym, v=p.nx, xs=p.nx, Ps=p.nsym)
    for k, c in comps.items():
        assert torch.equal(p.natural(b[k], c), p.natural(f[k], c)), k
    for k in ("obj", "g_loglik", "g_obj"):
        a, r = b[k].cpu().numpy(), f[k].cpu().numpy()
        assert np.abs(a - r).max() <= 1e-12 * max(np.abs(r).max(), 1e-300), k
    e_xs = rel_err(planes_T(p.natural(b["xs"], p.nx)), o["xs"])
    print(f"  xs vs oracle {e_xs:.1e}")
    assert e_xs <= TOL[dtype]
