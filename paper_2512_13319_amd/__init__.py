"""mapscan: parallel-in-time continuous-time MAP trajectory estimation on
MI355X (gfx950).

Thin Python layer over the C-ABI library `libmapscan.so` (include/mapscan.h):
it owns device memory through torch, passes raw pointers and the current HIP
stream, and wraps the fused scans in a `torch.autograd.Function`.  Every step
of the computation runs in the library's HIP kernels; there is no fallback,
so a missing library raises.

Layouts (see include/mapscan.h): the library reads and writes every
state-indexed array (measurements, step lengths, linearisation states, filter
and smoother moments) in a tiled layout whose tiles match the kernels'
64-lane x 16-state work units; `to_tiled` / `from_tiled` convert from / to
natural [components, n_states] planes.  Symmetric matrices are nx(nx+1)/2
lower-triangle components.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import _lib
from ._lib import MapError, MODELS

__all__ = ["Problem", "problem_from_workload", "filter_scan", "smoother_scan", "smooth",
           "two_filter_smooth", "autotune", "schedule", "lti_exact_terms",
           "iterated_nonlinear", "backward", "build_elements", "sym_to_full", "MapSmooth", "dense_output",
           "MapError", "N_THETA", "to_tiled", "from_tiled", "tiled_numel", "GraphedSmooth"]

N_THETA = {"linear": 0, "cv": 3, "vdp": 3, "lorenz63": 5, "ct": 4}
TILE = 1024      # states per tile: 64 lanes x 16 states
LANES, CHUNK = 64, 16


def n_tiles(n_states: int) -> int:
    return (n_states + TILE - 1) // TILE


def tiled_numel(n_states: int, comps: int) -> int:
    return n_tiles(n_states) * comps * TILE


def to_tiled(x: torch.Tensor) -> torch.Tensor:
    """[C, n_states] natural planes -> flat tiled buffer (zero padded)."""
    C, n = x.shape
    nt = n_tiles(n)
    xp = x.new_zeros(C, nt * TILE)
    xp[:, :n] = x
    return xp.view(C, nt, LANES, CHUNK).permute(1, 0, 3, 2).contiguous().view(-1)


def from_tiled(buf: torch.Tensor, comps: int, n_states: int) -> torch.Tensor:
    """flat tiled buffer -> [C, n_states] natural planes (a copy)."""
    nt = n_tiles(n_states)
    return buf[:nt * comps * TILE].view(nt, comps, CHUNK, LANES).permute(1, 0, 3, 2).reshape(
        comps, nt * TILE)[:, :n_states]


def steps_to_states(seg_off: np.ndarray, n_states: int, a: np.ndarray) -> np.ndarray:
    """Step-indexed [C, n_steps] -> state-indexed [C, n_states]: the value of
    the step that ends at each state; a segment's first state gets 0."""
    a = np.asarray(a, dtype=np.float64)
    n_steps = a.shape[-1]
    k = np.arange(n_steps)
    seg = np.searchsorted(seg_off, k, side="right") - 1
    out = np.zeros(a.shape[:-1] + (n_states,))
    out[..., k + seg + 1] = a
    return out


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def sym_to_full(planes: torch.Tensor, nx: int) -> torch.Tensor:
    """[nx(nx+1)/2, n] lower-triangle planes -> [n, nx, nx]."""
    n = planes.shape[1]
    out = planes.new_empty((n, nx, nx))
    c = 0
    for r in range(nx):
        for q in range(r + 1):
            out[:, r, q] = planes[c]
            out[:, q, r] = planes[c]
            c += 1
    return out


class Problem:
    """A batch of trajectories of one model, resident on the GPU.

    model     "cv" | "vdp" | "lorenz63" | "ct" | "linear"
    seg_off   int64 [n_seg+1] step offsets (host array or tensor)
    dt        [n_steps] step lengths (or a 0-d tensor / float for a shared value)
    y         [ny, n_steps] measurements
    m0, P0    [n_seg, nx], [n_seg, nx, nx] (or [nx], [nx, nx] shared)
    theta     [n_seg, n_theta] (or [n_theta] shared) model parameters
    xbar      [nx, n_states] linearisation states (nonlinear models)
    lin       dict of F, c, L, W, H, r, R for the linear model: each either one
              matrix or a leading per-step axis
    dtype     storage precision of every array (torch.float64 or torch.float32)
    arith     arithmetic precision: "f64" (default; with float32 storage this is
              the accurate FP32 mode) or "f32" (float32 storage only)
    chunk     schedule: states per lane (4, 8, 16, 32) or 0 for the library's choice
              (an autotuned one for this shape if `autotune` ran, else a
              heuristic)
    check_finite  every call waits for its stream and raises if a non-finite
              value was written (non-finite inputs, or a covariance that is not
              positive definite)
    om_divergence  minimise the Onsager--Machlup objective with its divergence
              term (a Newton step on it where it depends on the state); x*,
              P^s and the objective only (see MAP_OM_DIVERGENCE)
    n_sub     substeps per step (>= 2: each step is a block whose element is the
              element ODE integrated by n_sub Euler substeps; y is then
              [ny * n_sub, n_steps], component j * ny + c at the end of substep
              j + 1); see `dense_output`
    """

    def __init__(self, model, nx, ny, nw, seg_off, dt, y, m0, P0, theta=None, xbar=None, lin=None,
                 dtype=torch.float64, device="cuda", arith="f64", chunk=0, check_finite=False,
                 om_divergence=False, n_sub=1):
        _lib.load()
        self.n_sub = int(n_sub)
        self.chunk = int(chunk)
        self.check_finite = bool(check_finite)
        self.om_divergence = bool(om_divergence)
        self.model, self.nx, self.ny, self.nw = model, nx, ny, nw
        self.dtype, self.device = dtype, torch.device(device)
        if arith not in ("f64", "f32") or (arith == "f32" and dtype != torch.float32):
            raise ValueError("arith must be 'f64', or 'f32' with float32 storage")
        self.arith = arith
        t = lambda a: None if a is None else torch.as_tensor(a).to(self.device, dtype).contiguous()
        so = np.ascontiguousarray(np.asarray(seg_off if not torch.is_tensor(seg_off)
                                             else seg_off.cpu().numpy(), dtype=np.int64))
        self.seg_off_host = so
        self.seg_off = torch.as_tensor(so).to(self.device)
        self.n_seg = int(so.shape[0] - 1)
        self.n_steps = int(so[-1])
        self.n_states = self.n_steps + self.n_seg
        dt_np = np.asarray(dt.cpu().numpy() if torch.is_tensor(dt) else dt, dtype=np.float64).reshape(-1)
        if dt_np.size == 0:
            self.dt = t(np.ones(1))                       # no steps: any shared value
        elif dt_np.size == 1 or np.all(dt_np == dt_np[0]):
            self.dt = t(dt_np[:1])                        # one shared step length
        else:
            self.dt = to_tiled(t(steps_to_states(so, self.n_states, dt_np[None])))
        y_np = np.asarray(y.cpu().numpy() if torch.is_tensor(y) else y, dtype=np.float64)
        ny_all = ny * max(self.n_sub, 1)
        self.y = to_tiled(t(steps_to_states(so, self.n_states, y_np.reshape(ny_all, self.n_steps))))
        m0 = t(m0)
        P0 = t(P0)
        self.m0 = m0.reshape(-1, nx)
        self.P0 = P0.reshape(-1, nx, nx)
        self.n_theta = N_THETA[model]
        self.theta = None if theta is None else t(theta).reshape(-1, self.n_theta)
        self.xbar = None if xbar is None else to_tiled(t(xbar).reshape(nx, self.n_states))
        self.lin = None
        if lin is not None:
            self.lin = {}
            shapes = dict(F=(nx, nx), c=(nx,), L=(nx, nw), W=(nw, nw), H=(ny, nx), r=(ny,),
                          R=(ny, ny))
            for k, shp in shapes.items():
                a = t(lin[k])
                per_step = a.dim() == len(shp) + 1
                self.lin[k] = (a, int(np.prod(shp)) if per_step else 0)
        self._ws = None
        self._sync_struct()

    # ------------------------------------------------------------------ marshalling
    def _sync_struct(self):
        s = _lib.MapProblem()
        s.nx, s.ny, s.nw = self.nx, self.ny, self.nw
        s.dtype = (_lib.MAP_F64 if self.dtype == torch.float64 else
                   _lib.MAP_F32_FAST if self.arith == "f32" else _lib.MAP_F32)
        s.model = MODELS[self.model]
        s.n_theta = self.n_theta
        s.n_seg, s.n_steps = self.n_seg, self.n_steps
        s.chunk = self.chunk
        s.flags = ((_lib.MAP_CHECK_FINITE if self.check_finite else 0)
                   | (_lib.MAP_OM_DIVERGENCE if self.om_divergence else 0))
        s.n_sub = self.n_sub
        s.seg_off = self.seg_off.data_ptr()
        s.seg_off_host = self.seg_off_host.ctypes.data
        s.dt = self.dt.data_ptr()
        s.dt_stride = 0 if self.dt.numel() == 1 else 1
        s.y = self.y.data_ptr()
        s.m0 = self.m0.data_ptr()
        s.m0_stride = 0 if self.m0.shape[0] == 1 else self.nx
        s.P0 = self.P0.data_ptr()
        s.P0_stride = 0 if self.P0.shape[0] == 1 else self.nx * self.nx
        if self.theta is not None:
            s.theta = self.theta.data_ptr()
            s.theta_stride = 0 if self.theta.shape[0] == 1 else self.n_theta
        if self.xbar is not None:
            s.xbar = self.xbar.data_ptr()
        if self.lin is not None:
            for k in ("F", "c", "L", "W", "H", "r", "R"):
                a, st = self.lin[k]
                setattr(s, k, a.data_ptr())
                setattr(s, k + "_stride", st)
        self.struct = s

    def set_xbar(self, xbar):
        """xbar: natural [nx, n_states]."""
        self.xbar = to_tiled(xbar.to(self.device, self.dtype).reshape(self.nx, self.n_states))
        self._sync_struct()

    def set_theta(self, theta):
        self.theta = theta.to(self.device, self.dtype).reshape(-1, self.n_theta).contiguous()
        self._sync_struct()

    def workspace(self):
        lib = _lib.load()
        nbytes = lib.map_workspace_bytes(ctypes.byref(self.struct))
        if nbytes == 0:
            raise MapError(-2, lib.map_last_error().decode())
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _lib.check(lib.map_workspace_init(_ptr(self._ws), nbytes, _stream()))
        return self._ws

    # ------------------------------------------------------------------ allocation helpers
    @property
    def nsym(self):
        return self.nx * (self.nx + 1) // 2

    def _empty(self, *shape, dtype=None):
        return torch.empty(*shape, dtype=dtype or self.dtype, device=self.device)

    def _tiled(self, comps):
        """Uninitialised tiled buffer for a state-indexed output."""
        return self._empty(tiled_numel(self.n_states, comps))

    def natural(self, buf, comps):
        return None if buf is None else from_tiled(buf, comps, self.n_states)


def _nat(p, r, natural):
    """Replace tiled outputs by natural [C, n_states] planes when asked."""
    if not natural:
        return r
    comps = dict(S=p.nsym, v=p.nx, m=p.nx, P=p.nsym, xs=p.nx, Ps=p.nsym, xbar=p.nx)
    return {k: (p.natural(v, comps[k]) if (k in comps and v is not None) else v)
            for k, v in r.items()}


def problem_from_workload(wl, dtype=torch.float64, device="cuda", xbar=None, arith="f64",
                          chunk=0, check_finite=False, om_divergence=False):
    """Device-resident Problem from a `workloads.Workload`-like object."""
    return Problem(wl.model, wl.nx, wl.ny, wl.nw, wl.seg_off, wl.dt, wl.y, wl.m0, wl.P0,
                   theta=wl.theta if wl.model != "linear" else None, xbar=xbar,
                   lin=getattr(wl, "lin", None), dtype=dtype, device=device, arith=arith,
                   chunk=chunk, check_finite=check_finite, om_divergence=om_divergence,
                   n_sub=getattr(wl, "n_sub", 1))


def autotune(p: Problem, cache_path=None) -> int:
    """Time the fused step at every schedule (states per lane) on this problem
    and record the fastest for its shape; later calls with chunk = 0 use it.
    A nonlinear problem needs its linearisation point set (`set_xbar`).
    Returns the chosen chunk.  Synchronises the current stream."""
    lib = _lib.load()
    if p.chunk != 0:
        raise ValueError("autotune needs a Problem with chunk=0")
    ws = p.workspace()
    out = ctypes.c_int32(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _lib.check(lib.map_autotune(ctypes.byref(p.struct), _ptr(ws), ws.numel(), path,
                                ctypes.byref(out), _stream()))
    return int(out.value)


def lti_exact_terms(F, c, L, W, dt):
    """Terms (F~, c~, L~, W~ = I) of the library's one-step element that make it
    the exact discretisation of the time-invariant model dx/dt = F x + c + L w
    over a step dt (see map_lti_exact_terms).  Host numpy arrays in and out;
    use them as F, c, L, W of a "linear" Problem (nw = nx)."""
    lib = _lib.load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    nx, nw = F.shape[0], L.shape[1]
    c = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
    Ft = np.empty((nx, nx))
    ct = np.empty(nx)
    Lt = np.empty((nx, nx))
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    _lib.check(lib.map_lti_exact_terms(nx, nw, p(F), p(c), p(L), p(W), float(dt), p(Ft), p(ct),
                                       p(Lt)))
    return Ft, ct, Lt, np.eye(nx)


def schedule(p: Problem) -> int:
    """States per lane the scan entry points use for this problem."""
    lib = _lib.load()
    out = ctypes.c_int32(0)
    _lib.check(lib.map_schedule(ctypes.byref(p.struct), ctypes.byref(out)))
    return int(out.value)


def build_elements(p: Problem, natural=True):
    """Elements of every state as [A (nx*nx), b, C (sym), eta, J (sym)] components."""
    lib = _lib.load()
    n = p.nx * p.nx + 2 * p.nx + 2 * p.nsym
    out = p._tiled(n)
    _lib.check(lib.map_build_elements(ctypes.byref(p.struct), _ptr(out), _stream()))
    return p.natural(out, n) if natural else out


def filter_scan(p: Problem, moments=False, loglik=True, natural=True):
    lib = _lib.load()
    ws = p.workspace()
    S = p._tiled(p.nsym)
    v = p._tiled(p.nx)
    m = p._tiled(p.nx) if moments else None
    P = p._tiled(p.nsym) if moments else None
    ll = p._empty(p.n_seg, dtype=torch.float64) if loglik else None
    _lib.check(lib.map_filter_scan(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(m), _ptr(P),
                                   _ptr(ll), _ptr(ws), ws.numel(), _stream()))
    return _nat(p, dict(S=S, v=v, m=m, P=P, loglik=ll), natural)


def smoother_scan(p: Problem, S, v, covariances=True, objective=True, natural=True):
    """S, v: tiled buffers as returned by filter_scan(..., natural=False)."""
    lib = _lib.load()
    ws = p.workspace()
    xs = p._tiled(p.nx)
    Ps = p._tiled(p.nsym) if covariances else None
    obj = p._empty(p.n_seg, dtype=torch.float64) if objective else None
    _lib.check(lib.map_smoother_scan(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs),
                                     _ptr(Ps), _ptr(obj), _ptr(ws), ws.numel(), _stream()))
    return _nat(p, dict(xs=xs, Ps=Ps, obj=obj), natural)


def checkpoint_bytes(p: Problem) -> int:
    """Bytes of the filter checkpoint map_smooth_checkpointed writes for `p`."""
    n = int(_lib.load().map_checkpoint_bytes(ctypes.byref(p.struct)))
    if n == 0:
        _lib.check(-1)  # MAP_E_ARG, with the library's message
    return n


def smooth(p: Problem, covariances=True, loglik=True, objective=True, grad=False, out=None,
           natural=True, checkpoint=False):
    """Fused filter + trajectory scans (+ adjoint when grad).  `out` may carry
    preallocated tiled buffers (same keys as the result) to avoid allocations.
    With `checkpoint`, runs map_smooth_checkpointed: the result also holds the
    filter checkpoint (`ckpt`, a byte tensor) that `backward(..., ckpt=...)`
    rebuilds S, v from."""
    lib = _lib.load()
    ws = p.workspace()
    o = out or {}
    S = o.get("S") if o.get("S") is not None else p._tiled(p.nsym)
    v = o.get("v") if o.get("v") is not None else p._tiled(p.nx)
    xs = o.get("xs") if o.get("xs") is not None else p._tiled(p.nx)
    Ps = (o.get("Ps") if o.get("Ps") is not None else p._tiled(p.nsym)) \
        if covariances else None
    f64 = torch.float64
    ll = (o.get("loglik") if o.get("loglik") is not None else p._empty(p.n_seg, dtype=f64)) \
        if loglik else None
    obj = (o.get("obj") if o.get("obj") is not None else p._empty(p.n_seg, dtype=f64)) \
        if objective else None
    gl = gm = None
    if grad:
        gl = o.get("g_loglik") if o.get("g_loglik") is not None else p._empty(p.n_seg, p.n_theta, dtype=f64)
        gm = o.get("g_obj") if o.get("g_obj") is not None else p._empty(p.n_seg, p.n_theta, dtype=f64)
    if checkpoint:
        ck = o.get("ckpt") if o.get("ckpt") is not None else \
            torch.empty(checkpoint_bytes(p), dtype=torch.uint8, device=p.device)
        _lib.check(lib.map_smooth_checkpointed(
            ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs), _ptr(Ps), _ptr(ll), _ptr(obj),
            _ptr(gl), _ptr(gm), _ptr(ck), ck.numel(), _ptr(ws), ws.numel(), _stream()))
    else:
        ck = None
        _lib.check(lib.map_smooth(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs), _ptr(Ps),
                                  _ptr(ll), _ptr(obj), _ptr(gl), _ptr(gm), _ptr(ws), ws.numel(),
                                  _stream()))
    r = _nat(p, dict(S=S, v=v, xs=xs, Ps=Ps, loglik=ll, obj=obj, g_loglik=gl, g_obj=gm),
             natural)
    if ck is not None:
        r["ckpt"] = ck
    return r


def two_filter_smooth(p: Problem, covariances=True, loglik=True, out=None, natural=True):
    """Two-filter smoother (Sec. 4.3, eq. twofilter): filter scan, backward
    filter (reverse segmented scan of the later steps) and their per-state
    combination.  Same trajectory as `smooth`; `out` as there."""
    lib = _lib.load()
    ws = p.workspace()
    o = out or {}
    S = o.get("S") if o.get("S") is not None else p._tiled(p.nsym)
    v = o.get("v") if o.get("v") is not None else p._tiled(p.nx)
    xs = o.get("xs") if o.get("xs") is not None else p._tiled(p.nx)
    Ps = (o.get("Ps") if o.get("Ps") is not None else p._tiled(p.nsym)) \
        if covariances else None
    ll = (o.get("loglik") if o.get("loglik") is not None
          else p._empty(p.n_seg, dtype=torch.float64)) if loglik else None
    _lib.check(lib.map_two_filter_smooth(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs),
                                         _ptr(Ps), _ptr(ll), _ptr(ws), ws.numel(), _stream()))
    return _nat(p, dict(S=S, v=v, xs=xs, Ps=Ps, loglik=ll), natural)


def dense_output(p: Problem, S, v, xs, natural=True):
    """Sub-stepped blocks: filter and MAP state at the interior substeps of
    every block from tiled S, v, xs of `smooth` (natural=False).  Returns
    xd [(n_sub-1), nx, n_states], Sd [(n_sub-1), nsym, n_states],
    vd [(n_sub-1), nx, n_states] (natural) or the tiled buffers."""
    lib = _lib.load()
    k = p.n_sub - 1
    xd = p._tiled(p.nx * k)
    Sd = p._tiled(p.nsym * k)
    vd = p._tiled(p.nx * k)
    _lib.check(lib.map_dense_output(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs), _ptr(xd),
                                    _ptr(Sd), _ptr(vd), _stream()))
    if not natural:
        return dict(xd=xd, Sd=Sd, vd=vd)
    return dict(xd=p.natural(xd, p.nx * k).reshape(k, p.nx, p.n_states),
                Sd=p.natural(Sd, p.nsym * k).reshape(k, p.nsym, p.n_states),
                vd=p.natural(vd, p.nx * k).reshape(k, p.nx, p.n_states))


def iterated_nonlinear(p: Problem, n_iter: int, xbar0=None, covariances=True, loglik=True,
                       objective=True, grad=False, out=None, natural=True):
    """xbar0: natural [nx, n_states] or None (m0 of each segment).  `out` may
    carry preallocated tiled buffers (keys xbar, S, v, xs, Ps, loglik, obj,
    g_loglik, g_obj) to avoid allocations."""
    lib = _lib.load()
    ws = p.workspace()
    f64 = torch.float64
    o = out or {}
    get = lambda k, make: o[k] if o.get(k) is not None else make()
    xb = get("xbar", lambda: p._tiled(p.nx))
    S = get("S", lambda: p._tiled(p.nsym))
    v = get("v", lambda: p._tiled(p.nx))
    xs = get("xs", lambda: p._tiled(p.nx))
    Ps = get("Ps", lambda: p._tiled(p.nsym)) if covariances else None
    ll = get("loglik", lambda: p._empty(p.n_seg, dtype=f64)) if loglik else None
    obj = get("obj", lambda: p._empty(p.n_seg, dtype=f64)) if objective else None
    gl = get("g_loglik", lambda: p._empty(p.n_seg, p.n_theta, dtype=f64)) if grad else None
    gm = get("g_obj", lambda: p._empty(p.n_seg, p.n_theta, dtype=f64)) if grad else None
    x0 = None if xbar0 is None else to_tiled(xbar0.to(p.device, p.dtype))
    _lib.check(lib.map_iterated_nonlinear(ctypes.byref(p.struct), int(n_iter), _ptr(x0), _ptr(xb),
                                          _ptr(S), _ptr(v), _ptr(xs), _ptr(Ps), _ptr(ll),
                                          _ptr(obj), _ptr(gl), _ptr(gm), _ptr(ws), ws.numel(),
                                          _stream()))
    return _nat(p, dict(xbar=xb, S=S, v=v, xs=xs, Ps=Ps, loglik=ll, obj=obj, g_loglik=gl,
                        g_obj=gm), natural)


def elem_grad_size(p: Problem) -> int:
    """Values per part of map_backward's per-step element cotangents:
    A (nx*nx), b (nx), C (lower triangle) and R (lower triangle)."""
    return p.nx * p.nx + p.nx + p.nsym + p.ny * (p.ny + 1) // 2


def backward(p: Problem, S, v, covariances=True, objective=True, natural=True, loglik_grad=True,
             obj_grad=True, g_xs=None, elem_grads=False, ckpt=None, out=None):
    """Adjoint from saved (tiled) filter planes S, v: recomputes the trajectory
    and returns d loglik / d theta and d obj / d theta per segment (when
    asked), and with `g_xs` (a cotangent of x*: natural [nx, n_states] or a
    tiled buffer) d(l)/d theta by the implicit function theorem (`g_xs_theta`)
    together with mu = H^{-1} g_xs.  With `elem_grads`, also the per-step
    element cotangents (`g_elems`: natural [2 E, n_states] doubles, E =
    elem_grad_size(p): those of loglik then of obj, at the state each step
    ends at; a segment's first state is zero).  With `ckpt` (the filter
    checkpoint of smooth(..., checkpoint=True)) S, v are rebuilt instead of
    read: pass None for both (fresh buffers, returned as `S`, `v`) or tiled
    buffers to write.  `out` may carry preallocated tiled buffers for xs, Ps,
    obj, g_loglik and g_obj."""
    lib = _lib.load()
    ws = p.workspace()
    f64 = torch.float64
    if ckpt is not None:
        S = p._tiled(p.nsym) if S is None else S
        v = p._tiled(p.nx) if v is None else v
    o = out or {}

    def buf(key, make, want=True):
        return (o[key] if o.get(key) is not None else make()) if want else None
    xs = buf("xs", lambda: p._tiled(p.nx))
    Ps = buf("Ps", lambda: p._tiled(p.nsym), covariances)
    obj = buf("obj", lambda: p._empty(p.n_seg, dtype=f64), objective)
    gl = buf("g_loglik", lambda: p._empty(p.n_seg, p.n_theta, dtype=f64), loglik_grad)
    gm = buf("g_obj", lambda: p._empty(p.n_seg, p.n_theta, dtype=f64), obj_grad)
    gx = mu = vmu = gxt = None
    if g_xs is not None:
        g = g_xs.to(p.device, p.dtype)
        gx = to_tiled(g.reshape(p.nx, p.n_states)) if g.dim() == 2 else g.contiguous()
        mu = p._tiled(p.nx)
        vmu = p._tiled(p.nx)
        gxt = p._empty(p.n_seg, p.n_theta, dtype=f64)
    ge = None
    if elem_grads:
        ge = torch.zeros(tiled_numel(p.n_states, 2 * elem_grad_size(p)), dtype=f64,
                         device=p.device)
    _lib.check(lib.map_backward(ctypes.byref(p.struct), _ptr(S), _ptr(v), _ptr(xs), _ptr(Ps),
                                _ptr(obj), _ptr(gl), _ptr(gm), _ptr(gx), _ptr(mu), _ptr(vmu),
                                _ptr(gxt), _ptr(ge), _ptr(ckpt),
                                ckpt.numel() if ckpt is not None else 0, _ptr(ws), ws.numel(),
                                _stream()))
    r = _nat(p, dict(xs=xs, Ps=Ps, obj=obj, g_loglik=gl, g_obj=gm, mu=mu, g_xs_theta=gxt),
             natural)
    if ckpt is not None:
        r.update(_nat(p, dict(S=S, v=v), natural))
    if ge is not None:
        r["g_elems"] = from_tiled(ge, 2 * elem_grad_size(p), p.n_states) if natural else ge
    return r


class GraphedSmooth:
    """A launch sequence of `smooth` (form "rts"), of `two_filter_smooth`
    (form "two_filter"), of `iterated_nonlinear` from m0 with `n_iter`
    iterations (form "iterated") or of the checkpointed training step (form
    "checkpointed": `smooth(..., checkpoint=True)` for x*, the log-likelihood
    and the objective, then `backward` from the checkpoint for P^s and the
    gradients, into the same output keys) captured once into a HIP graph
    (torch.cuda.CUDAGraph on ROCm) with fixed output buffers, then replayed.
    Inputs are read from the Problem's device buffers at replay time, so
    refreshing their contents in place (same shapes) is seen by the next
    replay.  The sequence contains kernel launches only (the accumulators are
    cleared by a kernel, not by memset nodes)."""

    def __init__(self, p: Problem, covariances=True, loglik=True, objective=True, grad=False,
                 form="rts", n_iter=1):
        if form not in ("rts", "two_filter", "iterated", "checkpointed"):
            raise ValueError("form must be 'rts', 'two_filter', 'iterated' or 'checkpointed'")
        if form == "two_filter" and (objective or grad):
            raise ValueError("the two-filter form has no objective or gradients")
        if form == "checkpointed" and not grad:
            raise ValueError("the checkpointed form is a training step: grad=True")
        self.p = p
        f64 = torch.float64
        self.out = dict(S=p._tiled(p.nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx),
                        xbar=p._tiled(p.nx) if form == "iterated" else None,
                        Ps=p._tiled(p.nsym) if covariances else None,
                        loglik=p._empty(p.n_seg, dtype=f64) if loglik else None,
                        obj=p._empty(p.n_seg, dtype=f64) if objective else None,
                        g_loglik=p._empty(p.n_seg, p.n_theta, dtype=f64) if grad else None,
                        g_obj=p._empty(p.n_seg, p.n_theta, dtype=f64) if grad else None)
        kw = dict(covariances=covariances, loglik=loglik)
        if form == "checkpointed":
            self.out["ckpt"] = torch.empty(checkpoint_bytes(p), dtype=torch.uint8,
                                           device=p.device)

            def run():
                smooth(p, out=self.out, natural=False, covariances=False, loglik=loglik,
                       objective=objective, grad=False, checkpoint=True)
                backward(p, self.out["S"], self.out["v"], covariances=covariances,
                         objective=objective, natural=False, loglik_grad=grad, obj_grad=grad,
                         ckpt=self.out["ckpt"], out=self.out)
        elif form == "rts":
            def run():
                smooth(p, out=self.out, natural=False, objective=objective, grad=grad, **kw)
        elif form == "two_filter":
            def run():
                two_filter_smooth(p, out=self.out, natural=False, **kw)
        else:
            def run():
                iterated_nonlinear(p, n_iter, out=self.out, natural=False, objective=objective,
                                   grad=grad, **kw)
        p.workspace()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            run()   # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            run()

    def replay(self):
        self.graph.replay()
        return self.out


class MapSmooth(torch.autograd.Function):
    """(theta) -> (xs, loglik, obj) for a parametric model.

    The forward pass runs the fused scans with the adjoint enabled, so the
    gradients of loglik (Fisher identity) and obj (envelope theorem) with
    respect to theta come out of the same pass; backward scales them by the
    incoming cotangents.  A cotangent on xs (natural [nx, n_states]) goes
    through `map_backward`'s implicit-function VJP, which reads the filter
    planes S, v kept from the forward pass.  theta is [n_seg, n_theta]
    (per segment), or [n_theta] / [1, n_theta] shared by every segment (its
    gradient is then the sum over segments).  Nonlinear models are
    linearised about the problem's xbar, held fixed.  With `checkpoint`
    (third argument), only the filter checkpoint is kept instead of S, v
    (map_smooth_checkpointed), and a cotangent on xs rebuilds them from it."""

    @staticmethod
    def forward(ctx, theta, problem: Problem, checkpoint=False):
        problem.set_theta(theta.detach())
        r = smooth(problem, covariances=False, loglik=True, objective=True, grad=True,
                   natural=False, checkpoint=checkpoint)
        ctx.problem = problem
        ctx.checkpoint = bool(checkpoint)
        if checkpoint:
            kept = (r["ckpt"],)
        else:
            kept = (r["S"], r["v"])
        ctx.save_for_backward(r["g_loglik"], r["g_obj"], theta.detach().clone(), *kept)
        ctx.theta_shape = theta.shape
        ctx.theta_dtype = theta.dtype
        return problem.natural(r["xs"], problem.nx), r["loglik"], r["obj"]

    @staticmethod
    def backward(ctx, g_xs, g_ll, g_obj):
        gl, gm, theta, *kept = ctx.saved_tensors
        g = torch.zeros_like(gl)
        if g_ll is not None:
            g = g + g_ll[:, None] * gl
        if g_obj is not None:
            g = g + g_obj[:, None] * gm
        if g_xs is not None and bool((g_xs != 0).any()):
            p = ctx.problem
            p.set_theta(theta)   # the forward pass's theta (the problem may have moved on)
            if ctx.checkpoint:
                r = backward(p, None, None, covariances=False, objective=False, natural=False,
                             loglik_grad=False, obj_grad=False, g_xs=g_xs, ckpt=kept[0])
            else:
                r = backward(p, kept[0], kept[1], covariances=False, objective=False,
                             natural=False, loglik_grad=False, obj_grad=False, g_xs=g_xs)
            g = g + r["g_xs_theta"]
        if tuple(ctx.theta_shape) != tuple(g.shape):
            # one theta shared by every segment ([n_theta] or [1, n_theta])
            g = g.sum(0, keepdim=True)
        return g.to(ctx.theta_dtype).reshape(ctx.theta_shape), None, None
