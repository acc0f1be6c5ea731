"""The fused scans captured in a HIP graph: every replay, with eager work and
synchronisations in between, equals the eager result (and the oracle)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cref

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    import paper_2512_13319_amd as ms
    wl = workloads.cv_batched(n_seg=9, lmin=6.0, lmax=11.0, seed=77)
    p = ms.problem_from_workload(wl, dtype=torch.float64)
    eager = ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, natural=True)
    eager = {k: v.clone() for k, v in eager.items() if v is not None}
    # state-indexed outputs are tiled; only valid states are defined (the
    # padding of the last tile is never written)
    comps = dict(S=p.nsym, v=p.nx, xs=p.nx, Ps=p.nsym)

    def view(k, buf):
        return p.natural(buf, comps[k]) if k in comps else buf
    g = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=True)
    o = cref.smooth(wl)
    for rep in range(4):
        out = g.replay()
        torch.cuda.synchronize()
        for k, v in eager.items():
            assert torch.allclose(view(k, out[k]), v, rtol=1e-12, atol=1e-12), (rep, k)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
    xs = p.natural(out["xs"], p.nx).cpu().numpy().T
    assert np.abs(xs - o["xs"]).max() <= 1e-9 * np.abs(o["xs"]).max()
    assert np.abs(out["loglik"].cpu().numpy() - o["loglik"]).max() <= 1e-9 * np.abs(o["loglik"]).max()


def test_checkpointed_graph_replays_match_eager():
    """The checkpointed training step (forward call keeping the filter
    checkpoint, then the adjoint rebuilding S, v from it) captured in one
    graph: every replay equals the eager calls."""
    import paper_2512_13319_amd as ms
    wl = workloads.cv_batched(n_seg=9, lmin=8.0, lmax=12.5, seed=78)
    p = ms.problem_from_workload(wl, dtype=torch.float64, chunk=8)
    f = ms.smooth(p, covariances=False, loglik=True, objective=True, grad=False, natural=False,
                  checkpoint=True)
    b = ms.backward(p, None, None, covariances=True, objective=True, natural=False,
                    ckpt=f["ckpt"])
    torch.cuda.synchronize()
    comps = dict(S=p.nsym, v=p.nx, xs=p.nx, Ps=p.nsym)
    eager = {k: (p.natural(b[k], comps[k]) if k in comps else b[k]).clone()
             for k in ("S", "v", "xs", "Ps", "obj", "g_loglik", "g_obj")}
    eager["loglik"] = f["loglik"].clone()
    g = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=True,
                         form="checkpointed")
    for rep in range(4):
        out = g.replay()
        torch.cuda.synchronize()
        for k, v in eager.items():
            got = p.natural(out[k], comps[k]) if k in comps else out[k]
            assert torch.allclose(got, v, rtol=1e-12, atol=1e-12), (rep, k)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
