"""C-ABI checks that need no GPU: the library loads, exports every function
include/mapscan.h declares, and rejects bad arguments on the host before
launching anything.  Every call below is built to fail validation, so no
kernel is ever launched (device pointers are dummies)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2512_13319_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mapscan.h")

FAKE = 0x1000  # never dereferenced: validation fails first


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(map_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_lib.EXPORTS)
    v = int(re.search(r"#define MAPSCAN_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert lib.map_abi_version() == v


def test_struct_layout_matches_header():
    """The ctypes mirror lists the struct fields in header order."""
    txt = open(HEADER).read()
    body = txt[txt.index("typedef struct {"):txt.index("} map_problem;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"([A-Za-z_0-9]+)\s*[,;]", body)
    assert fields == [f for f, _ in _lib.MapProblem._fields_]


def good(seg_host):
    p = _lib.MapProblem()
    p.nx, p.ny, p.nw = 4, 2, 2
    p.dtype = _lib.MAP_F64
    p.model = _lib.MODELS["cv"]
    p.n_theta = 3
    p.n_seg = len(seg_host) - 1
    p.n_steps = int(seg_host[-1])
    p.seg_off = FAKE
    p.seg_off_host = seg_host.ctypes.data
    p.dt = FAKE
    p.dt_stride = 1
    p.y = FAKE
    p.m0, p.P0, p.theta = FAKE, FAKE, FAKE
    p.m0_stride, p.P0_stride, p.theta_stride = 4, 16, 3
    return p


def status_of(fn, *args):
    return fn(*args)


@pytest.fixture
def seg():
    return np.array([0, 100, 250], dtype=np.int64)


def test_workspace_bytes(seg):
    lib = _lib.load()
    p = good(seg)
    n = lib.map_workspace_bytes(ctypes.byref(p))
    assert n > 0
    p2 = good(seg)
    p2.dtype = _lib.MAP_F32          # FP32 storage, FP64 arithmetic: FP64 workspace
    assert lib.map_workspace_bytes(ctypes.byref(p2)) == n
    p2.dtype = _lib.MAP_F32_FAST     # FP32 arithmetic: FP32 workspace
    assert 0 < lib.map_workspace_bytes(ctypes.byref(p2)) < n
    p2.nx = 9
    assert lib.map_workspace_bytes(ctypes.byref(p2)) == 0
    assert b"outside" in lib.map_last_error()


def test_workspace_bytes_by_schedule(seg):
    """The workspace shrinks with more states per lane; chunk 0 (the library's
    choice) fits every schedule; other values are rejected."""
    lib = _lib.load()
    big = np.array([0, 5000, 12000], dtype=np.int64)   # 12002 states: 12, 24, 47 work tiles
    sizes = {}
    for c in (0, 4, 8, 16):
        p = good(big)
        p.chunk = c
        sizes[c] = lib.map_workspace_bytes(ctypes.byref(p))
    assert sizes[16] < sizes[8] < sizes[4] == sizes[0]
    p = good(seg)
    p.chunk = 5
    assert lib.map_workspace_bytes(ctypes.byref(p)) == 0
    assert b"chunk" in lib.map_last_error()
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1


def test_flags_are_validated(seg):
    """MAP_CHECK_FINITE and MAP_OM_DIVERGENCE are the known flags; other bits
    are rejected before any launch, and MAP_OM_DIVERGENCE rejects the
    log-likelihood, gradients, the adjoint entry point and the two-filter
    form."""
    lib = _lib.load()
    p = good(seg)
    p.flags = _lib.MAP_OM_DIVERGENCE
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, FAKE, FAKE, 1 << 40,
                               None) == -8
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, FAKE, None, FAKE,
                          1 << 40, None) == -8
    assert lib.map_two_filter_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE,
                                     1 << 40, None) == -8
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE, None, None,
                            None, None, None, None, None, 0, FAKE, 1 << 40, None) == -8
    assert b"MAP_OM_DIVERGENCE" in lib.map_last_error()
    assert "#define MAP_OM_DIVERGENCE %d" % _lib.MAP_OM_DIVERGENCE in open(HEADER).read()
    p.flags = 4
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1
    assert b"flags" in lib.map_last_error()
    p.flags = _lib.MAP_CHECK_FINITE
    assert lib.map_workspace_bytes(ctypes.byref(p)) > 0
    assert "#define MAP_CHECK_FINITE %d" % _lib.MAP_CHECK_FINITE in open(HEADER).read()


def test_autotune_validates_before_running(seg):
    lib = _lib.load()
    out = ctypes.c_int32(0)
    p = good(seg)
    assert lib.map_autotune(ctypes.byref(p), FAKE, 1 << 40, None, None, None) == -1
    assert lib.map_autotune(ctypes.byref(p), None, 1 << 40, None, ctypes.byref(out), None) == -7
    assert lib.map_autotune(ctypes.byref(p), FAKE, 16, None, ctypes.byref(out), None) == -7
    p.dtype = 9
    assert lib.map_autotune(ctypes.byref(p), FAKE, 1 << 40, None, ctypes.byref(out), None) == -3


@pytest.mark.parametrize("mutate,expect", [
    (lambda p: setattr(p, "dtype", 7), -3),
    (lambda p: setattr(p, "nx", 0), -2),
    (lambda p: setattr(p, "ny", 9), -2),
    (lambda p: setattr(p, "model", 17), -1),
    (lambda p: setattr(p, "n_theta", 2), -2),
    (lambda p: setattr(p, "n_seg", 0), -2),
    (lambda p: setattr(p, "seg_off", None), -1),
    (lambda p: setattr(p, "dt", None), -1),
    (lambda p: setattr(p, "dt_stride", 3), -1),
    (lambda p: setattr(p, "y", None), -1),
    (lambda p: setattr(p, "P0", None), -1),
    (lambda p: setattr(p, "theta", None), -1),
    (lambda p: setattr(p, "m0_stride", -4), -1),
    (lambda p: (setattr(p, "nx", 5), setattr(p, "ny", 2), setattr(p, "nw", 2)), -8),
])
def test_filter_rejects_bad_problem(seg, mutate, expect):
    lib = _lib.load()
    p = good(seg)
    mutate(p)
    st = lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40, None)
    assert st == expect, (st, lib.map_last_error())
    assert lib.map_last_error()


def test_layout_errors():
    lib = _lib.load()
    bad = np.array([0, 100, 50], dtype=np.int64)
    p = good(bad)
    p.n_steps = 50
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, None, None, FAKE,
                          1 << 40, None) == -4
    bad2 = np.array([1, 100, 250], dtype=np.int64)
    assert lib.map_smooth(ctypes.byref(good(bad2)), FAKE, FAKE, FAKE, None, None, None, None,
                          None, FAKE, 1 << 40, None) == -4
    seg = np.array([0, 100, 250], dtype=np.int64)
    p3 = good(seg)
    p3.n_steps = 251
    assert lib.map_smooth(ctypes.byref(p3), FAKE, FAKE, FAKE, None, None, None, None, None, FAKE,
                          1 << 40, None) == -4


def test_workspace_and_output_checks(seg):
    lib = _lib.load()
    p = good(seg)
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 16, None) == -7
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, None, 1 << 40,
                               None) == -7
    assert lib.map_filter_scan(ctypes.byref(p), None, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE, 1 << 40,
                               None) == -1
    assert lib.map_smoother_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                                 None) == -1
    # nothing to differentiate
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, None, None, None,
                            None, None, None, None, 0, FAKE, 1 << 40, None) == -1
    # a cotangent of x* needs mu, vmu and the output, none of them aliasing the inputs
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, None, FAKE, None,
                            FAKE + 64, FAKE + 128, None, None, 0, FAKE, 1 << 40, None) == -1
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE + 8, FAKE + 16, None, None, None, None,
                            FAKE + 24, FAKE + 16, FAKE + 32, FAKE + 40, None, None, 0, FAKE,
                            1 << 40, None) == -1
    assert b"distinct" in lib.map_last_error()
    # per-step element cotangents must not alias another buffer
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE + 8, FAKE + 16, None, None, None, None,
                            None, None, None, None, FAKE + 16, None, 0, FAKE, 1 << 40, None) == -1
    assert b"g_elems aliases" in lib.map_last_error()
    assert lib.map_iterated_nonlinear(ctypes.byref(p), 0, None, FAKE, FAKE, FAKE, FAKE, None, None,
                                      None, None, None, FAKE, 1 << 40, None) == -1
    assert lib.map_iterated_nonlinear(ctypes.byref(p), 2, None, FAKE, FAKE, FAKE, FAKE, None, None,
                                      None, None, None, FAKE, 1 << 40, None) == -1  # aliasing
    assert lib.map_build_elements(ctypes.byref(p), None, None) == -1
    assert lib.map_filter_scan(None, FAKE, FAKE, None, None, None, FAKE, 1 << 40, None) == -1


def work_tiles(n_states, chunk):
    ts = 64 * chunk
    full, rem = divmod(n_states, ts)
    return full if (full > 0 and 0 < rem <= 8) else -(-n_states // ts)


def test_checkpoint_size_and_arguments():
    """The filter checkpoint holds (S, v) -- nx(nx+1)/2 + nx values of the
    arithmetic type -- per block of four work tiles of the schedule the
    adjoint resolves; the checkpointed entry points reject a missing, short,
    aliased or workspace-overlapping checkpoint, and problems the adjoint
    does not take, before launching anything."""
    lib = _lib.load()
    big = np.array([0, 5000, 12000, 40000], dtype=np.int64)   # 40003 states
    ns = 40003
    for chunk in (4, 8, 16, 32):
        for dtype, size in ((_lib.MAP_F64, 8), (_lib.MAP_F32, 8), (_lib.MAP_F32_FAST, 4)):
            p = good(big)
            p.chunk, p.dtype = chunk, dtype
            blocks = -(-work_tiles(ns, chunk) // 4)
            assert lib.map_checkpoint_bytes(ctypes.byref(p)) == 14 * blocks * size
    p = good(big)
    p.chunk = 16
    need = lib.map_checkpoint_bytes(ctypes.byref(p))
    assert need == 14 * 10 * 8          # 40 work tiles of 1024 states, 10 blocks
    # the sizes the documentation quotes: 2^20 steps at 16 per lane (1024 work
    # tiles, the one-state tail merged), and the 4096-segment batch at 32
    one = good(np.array([0, 2 ** 20], dtype=np.int64))
    one.chunk = 16
    assert lib.map_checkpoint_bytes(ctypes.byref(one)) == 28672
    batch = good(np.array([0, 16224882 - 4095], dtype=np.int64))   # 16228978 states
    batch.n_seg, batch.n_steps = 4096, 16224882
    batch.seg_off_host = None
    batch.chunk, batch.dtype = 32, _lib.MAP_F32
    assert lib.map_checkpoint_bytes(ctypes.byref(batch)) == 1982 * 14 * 8
    bad = good(big)
    bad.nx = 9
    assert lib.map_checkpoint_bytes(ctypes.byref(bad)) == 0
    WS, CK = FAKE, FAKE + (1 << 41)      # a workspace of 2^40 bytes, the checkpoint past it

    def fwd(prob, ck, ck_bytes, S=FAKE + 8, ws_bytes=1 << 40):
        return lib.map_smooth_checkpointed(ctypes.byref(prob), S, FAKE + 16, FAKE + 24, None,
                                           None, None, FAKE + 32, None, ck, ck_bytes, WS,
                                           ws_bytes, None)

    assert fwd(p, None, need) == -1
    assert b"ckpt is NULL" in lib.map_last_error()
    assert fwd(p, CK, need - 1) == -1
    assert b"checkpoint has" in lib.map_last_error()
    assert fwd(p, CK, need, S=CK) == -1
    assert b"aliases" in lib.map_last_error()
    assert fwd(p, WS + 4096, need) == -1
    assert b"overlaps the workspace" in lib.map_last_error()
    assert fwd(p, CK, need, ws_bytes=16) == -7        # workspace too small: still checked
    lin = good(big)
    lin.model = _lib.MODELS["linear"]
    lin.n_theta = 0
    for k in ("F", "c", "L", "W", "H", "r", "R"):
        setattr(lin, k, FAKE)
    assert fwd(lin, CK, 1 << 30) == -8
    blk = good(big)
    blk.n_sub = 4
    assert fwd(blk, CK, 1 << 30) == -8

    def bwd(ck, ck_bytes, S=FAKE + 8, v=FAKE + 16, xs=FAKE + 24, g_obj=FAKE + 40):
        return lib.map_backward(ctypes.byref(p), S, v, xs, None, None, FAKE + 32, g_obj, None,
                                None, None, None, None, ck, ck_bytes, WS, 1 << 40, None)

    assert bwd(CK, need - 8) == -1
    assert b"checkpoint has" in lib.map_last_error()
    assert bwd(CK, need, v=FAKE + 8) == -1               # S and v are outputs: distinct
    assert b"S and v are outputs" in lib.map_last_error()
    assert bwd(CK, need, xs=FAKE + 16) == -1
    assert bwd(CK, need, g_obj=CK) == -1
    assert b"checkpoint aliases" in lib.map_last_error()
    assert bwd(WS + 256, need) == -1
    assert b"overlaps the workspace" in lib.map_last_error()


def test_gradients_need_parametric_model():
    lib = _lib.load()
    seg = np.array([0, 100], dtype=np.int64)
    p = good(seg)
    p.model = _lib.MODELS["linear"]
    p.n_theta = 0
    p.nx, p.ny, p.nw = 2, 1, 1
    for k in ("F", "c", "L", "W", "H", "r", "R"):
        setattr(p, k, FAKE)
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, FAKE, FAKE, FAKE,
                          1 << 40, None) == -8
    assert lib.map_backward(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE, FAKE, None, None,
                            None, None, None, None, 0, FAKE, 1 << 40, None) == -8
    p.R = None
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1


def test_nonlinear_model_needs_xbar():
    lib = _lib.load()
    seg = np.array([0, 100], dtype=np.int64)
    p = good(seg)
    p.model = _lib.MODELS["vdp"]
    p.nx, p.ny, p.nw = 2, 1, 2
    p.m0_stride, p.P0_stride = 2, 4
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1
    assert b"xbar" in lib.map_last_error()


def test_schedule_query():
    """map_schedule: the problem's own chunk when set; otherwise the library's
    heuristic, one of the four schedules."""
    lib = _lib.load()
    out = ctypes.c_int32(0)
    big = np.array([0, 5000, 12000], dtype=np.int64)
    for c in (4, 8, 16, 32):
        p = good(big)
        p.chunk = c
        assert lib.map_schedule(ctypes.byref(p), ctypes.byref(out)) == 0
        assert out.value == c
    p = good(big)
    assert lib.map_schedule(ctypes.byref(p), ctypes.byref(out)) == 0
    assert out.value in (4, 8, 16, 32)
    assert lib.map_schedule(ctypes.byref(p), None) == -1
    p.chunk = 3
    assert lib.map_schedule(ctypes.byref(p), ctypes.byref(out)) == -1


def test_lti_exact_terms_against_the_oracle():
    """The library's host-side exact discretisation (Taylor scaling and
    squaring, Jacobi) against the oracle's (scipy expm, eigh): same F~, c~ and
    L~ L~^T; argument errors are reported."""
    import paper_2512_13319_amd as ms
    from oracle import lti
    rng = np.random.default_rng(9)
    cases = [(np.array([[0.0, 1.0], [0.0, 0.0]]), np.zeros(2), np.array([[0.0], [1.0]]), 0.7 * np.eye(1), 1e-3),
             (np.array([[0.0, 1.0], [-0.5, -0.2]]), np.array([0.3, -0.1]), rng.normal(size=(2, 2)),
              np.eye(2), 0.05)]
    F4 = np.zeros((4, 4)); F4[:2, 2:] = np.eye(2); F4[2:, 2:] = -0.6 * np.eye(2)
    cases.append((F4, np.array([0, 0, 0.15, -0.1]), np.vstack([np.zeros((2, 2)), np.eye(2)]),
                  0.5 * np.eye(2), 0.08))
    for F, c, L, W, dt in cases:
        a = ms.lti_exact_terms(F, c, L, W, dt)
        b = lti.implicit_equivalent(F, c, L, W, dt)
        assert np.abs(a[0] - b[0]).max() <= 1e-11 * max(1.0, np.abs(b[0]).max())
        assert np.abs(a[1] - b[1]).max() <= 1e-11 * max(1.0, np.abs(b[1]).max())
        Ca, Cb = a[2] @ a[2].T, b[2] @ b[2].T
        assert np.abs(Ca - Cb).max() <= 1e-12 * np.abs(Cb).max()
    lib = _lib.load()
    F = np.eye(2)
    L = np.eye(2)
    out = np.empty(4)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    assert lib.map_lti_exact_terms(2, 2, p(F), None, p(L), p(L), 0.0, p(out), p(out), p(out)) == -1
    assert lib.map_lti_exact_terms(9, 2, p(F), None, p(L), p(L), 0.1, p(out), p(out), p(out)) == -2
    Fn = F.copy(); Fn[0, 0] = np.nan
    assert lib.map_lti_exact_terms(2, 2, p(Fn), None, p(L), p(L), 0.1, p(out), p(out), p(out)) == -5


def test_substep_blocks_are_validated(seg):
    """n_sub: [0, 64]; blocks are built for the constant-velocity model with
    nx = 4 and for Van der Pol in FP64 arithmetic, give no log-likelihood,
    objective, gradients, two-filter form or divergence term; the dense output
    needs blocks.  All rejected on the host."""
    lib = _lib.load()
    p = good(seg)
    p.n_sub = 65
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -1
    p.n_sub = 10
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, FAKE, FAKE, 1 << 40,
                               None) == -8
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE, None, None, FAKE,
                          1 << 40, None) == -8
    assert lib.map_two_filter_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE,
                                     1 << 40, None) == -8
    p.flags = _lib.MAP_OM_DIVERGENCE
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, None, None, FAKE,
                          1 << 40, None) == -8
    p.flags = 0
    p.dtype = _lib.MAP_F32_FAST
    assert lib.map_dense_output(ctypes.byref(p), FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -8
    p.dtype = _lib.MAP_F64
    p.model, p.nx, p.ny, p.nw, p.n_theta = _lib.MODELS["lorenz63"], 3, 3, 3, 5
    p.m0_stride, p.P0_stride, p.theta_stride = 3, 9, 5
    p.xbar = FAKE
    assert lib.map_dense_output(ctypes.byref(p), FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -8
    q = good(seg)
    q.n_sub = 1
    assert lib.map_dense_output(ctypes.byref(q), FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1


def test_general_linear_shapes_are_validated(seg):
    """The general linear model takes nx <= 8 with ny, nw <= nx (padded where
    no instantiation of its own exists); above nx = 4 it needs FP64 arithmetic
    and has no two-filter form."""
    lib = _lib.load()
    p = good(seg)
    p.model, p.n_theta = _lib.MODELS["linear"], 0
    p.nx, p.ny, p.nw = 6, 2, 3
    p.m0_stride, p.P0_stride = 6, 36
    for k in ("F", "c", "L", "W", "H", "r", "R"):
        setattr(p, k, FAKE)
    assert lib.map_workspace_bytes(ctypes.byref(p)) > 0
    p.dtype = _lib.MAP_F32_FAST
    assert lib.map_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, None, None, None, FAKE,
                          1 << 40, None) in (-7, -8)
    p.dtype = _lib.MAP_F64
    assert lib.map_two_filter_smooth(ctypes.byref(p), FAKE, FAKE, FAKE, None, None, FAKE,
                                     1 << 40, None) == -8
    p.ny = 7   # more measurements than states: no padded form
    assert lib.map_filter_scan(ctypes.byref(p), FAKE, FAKE, None, None, None, FAKE, 1 << 40,
                               None) == -8
