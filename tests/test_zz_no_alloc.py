"""map_smooth_noalloc (fixed device scratch, no caller workspace) against
map_smooth (caller-owned workspace), both called through the C-ABI: two calls
in a row, the second on a smaller problem, in FP64 and FP32 storage, with every
output of the fused step.  Also checks the oracle on the second call and the
host-side rejection of a problem whose workspace exceeds the scratch."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import cref

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-9, torch.float32: 1e-4}


def _outs(p):
    f64 = torch.float64
    return dict(S=p._tiled(p.nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx), Ps=p._tiled(p.nsym),
                loglik=p._empty(p.n_seg, dtype=f64), obj=p._empty(p.n_seg, dtype=f64),
                g_loglik=p._empty(p.n_seg, p.n_theta, dtype=f64),
                g_obj=p._empty(p.n_seg, p.n_theta, dtype=f64))


def _call(lib, p, o, noalloc):
    import paper_2512_13319_amd as ms
    P = ms._ptr
    args = [ctypes.byref(p.struct), P(o["S"]), P(o["v"]), P(o["xs"]), P(o["Ps"]), P(o["loglik"]),
            P(o["obj"]), P(o["g_loglik"]), P(o["g_obj"])]
    if noalloc:
        st = lib.map_smooth_noalloc(*args, ms._stream())
    else:
        ws = p.workspace()
        st = lib.map_smooth(*args, P(ws), ws.numel(), ms._stream())
    assert st == 0, lib.map_last_error()


def _rel(a, b):
    a = a.double().cpu().numpy().reshape(a.shape[0], -1)
    b = b.double().cpu().numpy().reshape(b.shape[0], -1)
    scale = np.maximum(np.abs(b).max(axis=1, keepdims=True), 1e-300)
    return float((np.abs(a - b) / scale).max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_map_smooth_twice(dtype):
    import paper_2512_13319_amd as ms
    from paper_2512_13319_amd import _lib
    lib = _lib.load()
    cases = [workloads.cv_batched(n_seg=5, lmin=9.0, lmax=12.0, seed=41),
             workloads.cv_batched(n_seg=2, lmin=6.0, lmax=9.0, seed=42)]
    for n, wl in enumerate(cases):
        p = ms.problem_from_workload(wl, dtype=dtype)
        print("noalloc case", n, dtype, "n_states", p.n_states, flush=True)
        ref = _outs(p)
        got = _outs(p)
        _call(lib, p, ref, noalloc=False)
        _call(lib, p, got, noalloc=True)
        torch.cuda.synchronize()
        comps = dict(S=p.nsym, v=p.nx, xs=p.nx, Ps=p.nsym)
        for k in ref:
            a, b = got[k], ref[k]
            if k in comps:
                a, b = p.natural(a, comps[k]), p.natural(b, comps[k])
            if k in ("loglik", "obj"):
                a, b = a[None], b[None]
            err = _rel(a, b)
            assert err <= TOL[dtype], (n, k, err)
        o = cref.smooth(wl)
        xs = p.natural(got["xs"], p.nx).double().cpu().numpy().T
        e = np.abs(xs - o["xs"]).max(0) / np.abs(o["xs"]).max(0)
        assert e.max() <= (1e-9 if dtype == torch.float64 else 2e-4), e


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    """A 2^23-step problem needs more than the 64 MiB scratch: rejected on the
    host (MAP_E_WORKSPACE) before anything is launched."""
    from paper_2512_13319_amd import _lib
    lib = _lib.load()
    seg = np.array([0, 1 << 23], dtype=np.int64)
    p = _lib.MapProblem()
    p.nx, p.ny, p.nw = 4, 2, 2
    p.dtype = _lib.MAP_F64
    p.model = _lib.MODELS["cv"]
    p.n_theta = 3
    p.n_seg, p.n_steps = 1, int(seg[-1])
    fake = 0x1000
    p.seg_off, p.seg_off_host = fake, seg.ctypes.data
    p.dt, p.dt_stride, p.y = fake, 0, fake
    p.m0, p.P0, p.theta = fake, fake, fake
    st = lib.map_smooth_noalloc(ctypes.byref(p), fake, fake, fake, None, None, None, None, None,
                                None)
    assert st == -7, lib.map_last_error()
    assert b"scratch" in lib.map_last_error()
