"""ctypes front end of the plain-C sequential oracle `kfs.c` (test
infrastructure only; the product path never imports this).

`smooth(wl, xbar)` solves the discretised linear-affine MAP problem of every
segment of a `workloads.Workload`, linearised about `xbar` (states, [nx,
n_states]) for nonlinear models, with the covariance-form Kalman filter and
the discrete RTS smoother (Sec. 2.5, Sec. 4.3).  `iterate(wl)` runs the
iterated linearisation of Sec. 4.4 from xbar^(0) = m0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import models

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libkfs.so")
_lib = None


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-shared", "-fPIC",
                               os.path.join(_HERE, "kfs.c"), "-lm", "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
        _lib.oracle_smooth.restype = ctypes.c_long
    return _lib


def native_lib(out_dir: str):
    """The same oracle compiled for the host it runs on (gcc -O3
    -march=native, no fast-math: the arithmetic is the same IEEE arithmetic)
    into `out_dir`, for timing it as a CPU baseline.  Returns the loaded
    library, to pass as `lib=` to `smooth` / `iterate`."""
    os.makedirs(out_dir, exist_ok=True)
    so = os.path.join(out_dir, "libkfs_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-D_DEFAULT_SOURCE",
                           "-shared", "-fPIC", os.path.join(_HERE, "kfs.c"), "-lm", "-o", so])
    lib = ctypes.CDLL(so)
    lib.oracle_smooth.restype = ctypes.c_long
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _terms(wl, xbar):
    """Per-step (or per-segment) model terms in the C oracle's layout."""
    nx, ny, nw = wl.nx, wl.ny, wl.nw
    S, N = wl.n_seg, wl.n_steps
    if wl.model == "linear":
        lin = wl.lin
        return dict(F=(lin["F"], nx * nx, 0), c=(lin["c"], nx, 0), L=(lin["L"], 0, 0),
                    W=(lin["W"], 0, 0), H=(lin["H"], ny * nx, 0), r=(lin["r"], ny, 0),
                    R=(lin["R"], 0, 0))
    if wl.model == "cv":
        F = np.empty((S, nx, nx)); c = np.zeros((1, nx)); Wm = np.empty((S, nw, nw))
        R = np.empty((S, ny, ny))
        for s in range(S):
            F_, _, L, W_, H, _, R_ = models.terms_numpy("cv", wl.theta[s], np.zeros((1, nx)), nx)
            F[s], Wm[s], R[s] = F_[0], W_, R_
        return dict(F=(F, 0, nx * nx), c=(c, 0, 0), L=(np.ascontiguousarray(L), 0, 0),
                    W=(Wm, 0, nw * nw), H=(np.ascontiguousarray(H[0]), 0, 0),
                    r=(np.zeros((1, ny)), 0, 0), R=(R, 0, ny * ny))
    F = np.empty((N, nx, nx)); c = np.empty((N, nx)); H = np.empty((N, ny, nx))
    r = np.empty((N, ny)); Wm = np.empty((S, nw, nw)); R = np.empty((S, ny, ny))
    L = None
    Ls = []
    for s in range(S):
        st = wl.seg_steps(s)
        xb = xbar[:, st.start + s + 1: st.stop + s + 1].T
        F_, c_, L, W_, H_, r_, R_ = models.terms_numpy(wl.model, wl.theta[s], xb, nx,
                                                       wl.y[:, st].T)
        Ls.append(L)
        F[st], c[st], H[st], r[st], Wm[s], R[s] = F_, c_, H_, r_, W_, R_
    # L may depend on the segment's parameters (ct)
    Lall = np.ascontiguousarray(np.stack(Ls))
    return dict(F=(F, nx * nx, 0), c=(c, nx, 0), L=(Lall, 0, nx * nw),
                W=(Wm, 0, nw * nw), H=(H, ny * nx, 0), r=(r, ny, 0), R=(R, 0, ny * ny))


def smooth(wl, xbar=None, lib=None):
    """Returns dict(m [n_states,nx], P [n_states,nx,nx], xs, Ps, loglik [n_seg], mstar [n_seg])."""
    lib = lib or _load()
    nx, ny, nw = wl.nx, wl.ny, wl.nw
    S = wl.n_seg
    NS = wl.n_states
    if xbar is None:
        xbar = np.zeros((nx, NS))
    t = _terms(wl, xbar)
    keep = []

    def arg(key):
        a, st, sg = t[key]
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return [_p(a), ctypes.c_long(st), ctypes.c_long(sg)]

    seg_off = np.ascontiguousarray(wl.seg_off, dtype=np.int64)
    dt = np.ascontiguousarray(wl.dt, dtype=np.float64)
    y = np.ascontiguousarray(wl.y.T, dtype=np.float64)
    m0 = np.ascontiguousarray(wl.m0, dtype=np.float64)
    P0 = np.ascontiguousarray(wl.P0, dtype=np.float64)
    m = np.empty((NS, nx)); P = np.empty((NS, nx, nx))
    xs = np.empty((NS, nx)); Ps = np.empty((NS, nx, nx))
    ll = np.empty(S); ms = np.empty(S)
    args = [ctypes.c_int(nx), ctypes.c_int(ny), ctypes.c_int(nw), ctypes.c_long(S), _p(seg_off)]
    for key in ("F", "c", "L", "W", "H", "r", "R"):
        args += arg(key)
    args += [_p(dt), _p(y), _p(m0), ctypes.c_long(nx), _p(P0), ctypes.c_long(nx * nx),
             _p(m), _p(P), _p(xs), _p(Ps), _p(ll), _p(ms)]
    rc = lib.oracle_smooth(*args)
    if rc != S:
        raise FloatingPointError("oracle: segment %d lost positive definiteness" % (-rc - 1))
    return dict(m=m, P=P, xs=xs, Ps=Ps, loglik=ll, mstar=ms)


def iterate(wl, n_iter=None, xbar0=None, keep_iterates=False, lib=None):
    """Iterated linearisation (Sec. 4.4) from xbar^(0) = m0 at every state.
    Returns the last solve's outputs (with 'xbar' = its linearisation point)
    and optionally every iterate [n_iter, nx, n_states]."""
    n_iter = wl.n_iter if n_iter is None else n_iter
    if xbar0 is None:
        xbar = np.empty((wl.nx, wl.n_states))
        for s in range(wl.n_seg):
            xbar[:, wl.seg_states(s)] = wl.m0[s][:, None]
    else:
        xbar = xbar0
    its = []
    out = None
    for _ in range(n_iter):
        out = smooth(wl, xbar, lib=lib)
        out["xbar"] = xbar
        xbar = out["xs"].T.copy()
        if keep_iterates:
            its.append(xbar)
    if keep_iterates:
        out["iterates"] = np.stack(its)
    return out


def two_filter(wl, xbar=None, suffix=False):
    """Two-filter smoother (Sec. 4.3, eq. twofilter) of every segment, from the
    forward filter of `smooth` and the conditional value function of the steps
    after each state (see `oracle_two_filter` in kfs.c).  Returns dict(xs,
    Ps, m, P) and, with suffix=True, the run after each state as
    suf = dict(A, b, C, eta, J) with leading dimension n_states."""
    lib = _load()
    nx, ny, nw = wl.nx, wl.ny, wl.nw
    S = wl.n_seg
    NS = wl.n_states
    if xbar is None:
        xbar = np.zeros((nx, NS))
    fw = smooth(wl, xbar)
    t = _terms(wl, xbar)
    keep = []

    def arg(key):
        a, st, sg = t[key]
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return [_p(a), ctypes.c_long(st), ctypes.c_long(sg)]

    seg_off = np.ascontiguousarray(wl.seg_off, dtype=np.int64)
    dt = np.ascontiguousarray(wl.dt, dtype=np.float64)
    y = np.ascontiguousarray(wl.y.T, dtype=np.float64)
    m = np.ascontiguousarray(fw["m"]); P = np.ascontiguousarray(fw["P"])
    xs = np.empty((NS, nx)); Ps = np.empty((NS, nx, nx))
    suf = np.empty((NS, 3 * nx * nx + 2 * nx)) if suffix else None
    args = [ctypes.c_int(nx), ctypes.c_int(ny), ctypes.c_int(nw), ctypes.c_long(S), _p(seg_off)]
    for key in ("F", "c", "L", "W", "H", "r", "R"):
        args += arg(key)
    args += [_p(dt), _p(y), _p(m), _p(P), _p(xs), _p(Ps),
             _p(suf) if suffix else ctypes.c_void_p(None)]
    lib.oracle_two_filter.restype = ctypes.c_long
    rc = lib.oracle_two_filter(*args)
    if rc != S:
        raise FloatingPointError("oracle: segment %d has a singular two-filter system" % (-rc - 1))
    out = dict(xs=xs, Ps=Ps, m=fw["m"], P=fw["P"])
    if suffix:
        n2 = nx * nx
        out["suf"] = dict(A=suf[:, :n2].reshape(NS, nx, nx), b=suf[:, n2:n2 + nx],
                          C=suf[:, n2 + nx:2 * n2 + nx].reshape(NS, nx, nx),
                          eta=suf[:, 2 * n2 + nx:2 * n2 + 2 * nx],
                          J=suf[:, 2 * n2 + 2 * nx:].reshape(NS, nx, nx))
    return out
