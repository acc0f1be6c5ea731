#!/usr/bin/env python
"""Throughput of the parallel-in-time MAP smoother on one MI355X.

One step = one pass of the whole hot path over the workload resident in HBM:
filter scan (information form), trajectory scan with smoothed covariances,
log-likelihood and objective, and the fused adjoint (gradients of both with
respect to the constant-velocity parameters gamma, q, r).  The default
workload is the 2-D constant-velocity tracking SDE with nx = 4, ny = 2,
T = 2^20 uniform steps (dt = 1e-3), one trajectory.

Prints one JSON line.  Kernel durations for the roofline come from HIP events
the library records around each launch on its stream during the timed loop.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "smoothed time-steps/sec (fwd+adjoint) at nx=4, T=2^20, vs plain scan; % HBM peak"
HBM_PEAK_GBS = 8000.0
# both storage modes compute in FP64 (FP32 storage is converted on load), so
# the FP64 vector peak applies to either
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 78.6}


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def library_source_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2512_13319_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def schedule_info(chunk, tuned):
    """The schedule a run used: a flat one (states per lane) or the
    segment-local one (one wavefront per segment)."""
    if chunk > 0:
        return {"kind": "flat", "states_per_lane": chunk, "autotuned": tuned}
    return {"kind": "wavefront per segment", "states_per_lane": None, "autotuned": tuned}


def counter_record(dtype, workload="cv4_T2p20"):
    """Per-launch counter figures of the scan kernels on a workload
    (rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a device-copy calibration,
    SQ_INSTS_VALU_FLOPS_FP64 checked against a multiply of known size), and
    whether they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters_%s_%s.json" % (workload, dtype))
    if not os.path.exists(path):
        return None, False
    with open(path) as fh:
        rec = json.load(fh)
    return rec, rec.get("source_sha256_16") == library_source_hash()


def kernel_bytes(nx, ny, s, kind):
    """Algorithmic HBM bytes per state of each pass (each input read once,
    each output written once; the pass-to-pass intermediate S, v counted once
    as written by the filter and once as read by the trajectory pass)."""
    sym = nx * (nx + 1) // 2
    return {
        "filter_up": ny * s,                              # read y
        "fused_down": (ny + sym + nx) * s,                # read y, write S, v
        "traj_down": (sym + nx + ny + nx + sym) * s,      # read S, v, y; write xs, Ps
        "traj_down_adjoint": (sym + nx + ny + nx + sym) * s,
        "two_filter_up": (ny + sym + nx) * s,             # read y, write S, v
        "two_filter_down": (sym + nx + ny + nx + sym) * s,  # read S, v, y; write xs, Ps
        # segment-local schedule: the whole step in one kernel
        "seg_wave": (ny + 2 * (sym + nx) + nx + sym) * s,
    }[kind]


def roofline_for(kern, rec, fresh, n_states, nx, ny, s, dtype, schedule=None):
    """Roofline object of the longest kernel in `kern` {name: (count, ms)}.

    The bound is the roof the kernel's arithmetic intensity puts it under:
    counted FP64 flops per algorithmic HBM byte against the ridge point
    78.6 TFLOP/s / 8 TB/s (9.8 flop/B). Below the ridge the kernel is priced
    against HBM with its algorithmic bytes, above it against the FP64 vector
    roof with its counted flops. Without a flop count for this workload, or
    with one taken at another schedule (states per lane: the per-state work of
    the scans depends on it), it is priced against HBM."""
    dom = max((k for k in kern if k != "aux"), key=lambda k: kern[k][1])
    dom_ms = kern[dom][1]
    bytes_state = kernel_bytes(nx, ny, s, dom)
    bytes_dom = bytes_state * n_states
    hbm_gbs = bytes_dom / (dom_ms * 1e-3) / 1e9
    kc = (rec or {}).get("kernels", {}).get(dom)
    rec_sched = (rec or {}).get("states_per_lane")
    same_sched = schedule is None or rec_sched is None or rec_sched == schedule
    counted = kc is not None and kc.get("n_states") == n_states and same_sched
    ridge = VALU_PEAK_TFLOPS[dtype] * 1e3 / HBM_PEAK_GBS
    intensity = kc["flops_fp64_per_state"] / bytes_state if counted else None
    if counted and intensity >= ridge:
        # FP64 VALU roof: the per-state flop count of the kernel (counted, see
        # the counter record) over its measured launch duration
        flops = kc["flops_fp64_per_state"] * n_states
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS[dtype],
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS[dtype], 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    roof["traffic"] = kc["hbm_bytes"] if counted and fresh else None
    if counted:
        roof.update({"flops_per_state": kc["flops_fp64_per_state"],
                     "intensity_flop_per_byte": round(intensity, 2),
                     "ridge_flop_per_byte": round(ridge, 2),
                     "fp64_achieved_TFLOPs": round(kc["flops_fp64_per_state"] * n_states
                                                   / (dom_ms * 1e-3) / 1e12, 3),
                     "counters_current": fresh})
    if not same_sched:
        roof["counters_schedule"] = {"profiled": rec_sched, "measured": schedule}
    roof.update({
        "kernel": dom, "kernel_ms": round(dom_ms, 4),
        "kernels_ms": {k: round(v[1], 4) for k, v in kern.items()},
        "hbm_algorithmic": {"bytes": bytes_dom, "achieved_GBs": round(hbm_gbs, 1),
                            "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}})
    return roof


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"],
                    help="storage type of inputs and outputs (arithmetic is FP64 in both)")
    ap.add_argument("--log2T", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=2048,
                    help="steps of the autograd-oracle sample (the C oracle runs the whole track)")
    ap.add_argument("--cpu-sample-ct", type=int, default=64,
                    help="tracks of the coordinated-turn CPU-baseline sample")
    ap.add_argument("--cpu-reps", type=int, default=5,
                    help="timed runs of each C-oracle baseline (median reported)")
    ap.add_argument("--cpu-batched-segs", type=int, default=1024,
                    help="segments of the batched one-thread C-oracle baseline (the thread-pool "
                         "run takes all 4096); 0: all")
    ap.add_argument("--cpu-sample-tf", type=int, default=2 ** 20,
                    help="steps of the two-filter CPU-baseline sample")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default schedule instead of autotuning it")
    ap.add_argument("--no-two-filter", action="store_true",
                    help="skip the two-filter smoother measurement")
    ap.add_argument("--no-checkpointed", action="store_true",
                    help="skip the checkpointed training step (filter checkpoint, adjoint "
                         "rebuilds S, v)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-storage run of the headline step")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact-discretisation (linear-model path) measurement")
    ap.add_argument("--ct-chunk", type=int, default=0,
                    help="states per lane for the coordinated-turn solve (0: autotuned, or the "
                         "library's heuristic with --no-autotune)")
    ap.add_argument("--no-ct", action="store_true",
                    help="skip the coordinated-turn (iterated nonlinear) measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched ragged-segment measurement (4096 segments)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: the library runs each scan on one MI355X "
              "(multi-GPU sharding is a design note only); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2512_13319_amd as ms
    import workloads
    from paper_2512_13319_amd import _lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    T = 2 ** args.log2T
    wl = workloads.cv(T=T, d=2, dt=1e-3, q=0.5, r=0.05, m0=[5, 5, 0, 0], P0=1e-2 * np.eye(4),
                      seed=2, name="cfg2_cv2d")
    p = ms.problem_from_workload(wl, dtype=tdt, device=dev)
    # schedule (states per lane) picked by the library's autotuner, untimed
    tuned = not args.no_autotune
    if tuned:
        ms.autotune(p)
    chunk = ms.schedule(p)
    nsym = p.nsym
    out = dict(S=p._tiled(nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx), Ps=p._tiled(nsym),
               loglik=p._empty(1, dtype=torch.float64), obj=p._empty(1, dtype=torch.float64),
               g_loglik=p._empty(1, 3, dtype=torch.float64), g_obj=p._empty(1, 3, dtype=torch.float64))
    lib = _lib.load()

    def step_fwdadj():
        ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, out=out,
                  natural=False)

    def step_plain():
        ms.smooth(p, covariances=True, loglik=False, objective=False, grad=False, out=out,
                  natural=False)

    def timed(fn, steps, warmup, profile):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        if profile:
            _lib.check(lib.map_profile_enable(steps * 8))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_step = e0.elapsed_time(e1) / steps
        kern = {}
        if profile:
            import ctypes
            for name, kind in _lib.PROF_KINDS.items():
                c = ctypes.c_int64()
                tot = ctypes.c_double()
                _lib.check(lib.map_profile_read(kind, ctypes.byref(c), ctypes.byref(tot)))
                if c.value:
                    kern[name] = (c.value, tot.value / c.value)
            _lib.check(lib.map_profile_enable(0))
        return ms_step, wall / steps * 1e3, kern

    # per-kernel durations: HIP events recorded by the library around each launch
    ms_fa_e, wall_fa_e, kern_fa = timed(step_fwdadj, args.steps, args.warmup, True)
    ms_pl_e, wall_pl_e, kern_pl = timed(step_plain, args.steps, args.warmup, True)
    # headline: the same launch sequence captured once in a HIP graph and replayed
    if args.no_graph:
        ms_fa, wall_fa, ms_pl = ms_fa_e, wall_fa_e, ms_pl_e
    else:
        g_fa = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=True)
        ms_fa, wall_fa, _ = timed(g_fa.replay, args.steps, args.warmup, False)
        g_pl = ms.GraphedSmooth(p, covariances=True, loglik=False, objective=False, grad=False)
        ms_pl, _, _ = timed(g_pl.replay, args.steps, args.warmup, False)

    s = 8 if args.dtype == "f64" else 4
    step_bytes = (p.ny + 2 * (nsym + p.nx) + p.nx + nsym) * s * p.n_states
    rec, fresh = counter_record(args.dtype)
    # dominant kernel of the fwd+adjoint step
    roofline = roofline_for(kern_fa, rec, fresh, p.n_states, p.nx, p.ny, s, args.dtype, chunk)
    roofline["step_hbm_frac"] = round(step_bytes / (ms_fa * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    two_filter = None
    if not args.no_two_filter:
        # the two-filter smoother (Sec. 4.3) on the same workload: x*, P^s and
        # the log-likelihood (it has no objective or adjoint)
        tf_out = dict(S=out["S"], v=out["v"], xs=out["xs"], Ps=out["Ps"], loglik=out["loglik"])

        def step_tf():
            ms.two_filter_smooth(p, covariances=True, loglik=True, out=tf_out, natural=False)

        ms_tf_e, _, kern_tf = timed(step_tf, args.steps, args.warmup, True)
        if args.no_graph:
            ms_tf = ms_tf_e
        else:
            g_tf = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=False, grad=False,
                                    form="two_filter")
            ms_tf, _, _ = timed(g_tf.replay, args.steps, args.warmup, False)
        two_filter = {"value": T / (ms_tf * 1e-3), "unit": "time-steps/s", "ms_per_step": ms_tf,
                      "eager_ms_per_step": round(ms_tf_e, 4),
                      "outputs": "filter S, v; smoothed x*, P^s; log-likelihood",
                      "roofline": roofline_for(kern_tf, rec, fresh, p.n_states, p.nx, p.ny, s,
                                               args.dtype, chunk)}

    fp32 = None
    if args.dtype == "f64" and not args.no_fp32:
        # the headline step with FP32 storage of inputs and outputs (FP64
        # arithmetic and workspace), on the same track rounded to FP32
        p32 = ms.problem_from_workload(wl, dtype=torch.float32, device=dev)
        if tuned:
            ms.autotune(p32)
        out32 = dict(S=p32._tiled(nsym), v=p32._tiled(p32.nx), xs=p32._tiled(p32.nx),
                     Ps=p32._tiled(nsym), loglik=p32._empty(1, dtype=torch.float64),
                     obj=p32._empty(1, dtype=torch.float64),
                     g_loglik=p32._empty(1, 3, dtype=torch.float64),
                     g_obj=p32._empty(1, 3, dtype=torch.float64))

        def step_fa32():
            ms.smooth(p32, covariances=True, loglik=True, objective=True, grad=True, out=out32,
                      natural=False)

        ms_32_e, _, kern_32 = timed(step_fa32, args.steps, args.warmup, True)
        if args.no_graph:
            ms_32 = ms_32_e
        else:
            g_32 = ms.GraphedSmooth(p32, covariances=True, loglik=True, objective=True,
                                    grad=True)
            ms_32, _, _ = timed(g_32.replay, args.steps, args.warmup, False)
        fp32 = {"value": T / (ms_32 * 1e-3), "unit": "time-steps/s", "ms_per_step": ms_32,
                "eager_ms_per_step": round(ms_32_e, 4), "storage": "f32",
                "arithmetic": "f64",
                "schedule": schedule_info(ms.schedule(p32), tuned),
                "kernels_ms": {k: round(v[1], 4) for k, v in kern_32.items()}}

    checkpointed = None
    if not args.no_checkpointed:
        # the same training step with activation checkpointing: the forward
        # call keeps only the filter's block carries, the adjoint rebuilds S, v
        # from them (one more filter up-sweep without its cross-block step and
        # one more fused fix-up) before the trajectory pass with the gradients
        ck_out = dict(out)
        ck_out["ckpt"] = torch.empty(ms.checkpoint_bytes(p), dtype=torch.uint8, device=dev)

        def step_ck():
            ms.smooth(p, covariances=False, loglik=True, objective=True, grad=False, out=ck_out,
                      natural=False, checkpoint=True)
            ms.backward(p, ck_out["S"], ck_out["v"], covariances=True, objective=True,
                        natural=False, ckpt=ck_out["ckpt"], out=ck_out)

        ms_ck_e, _, kern_ck = timed(step_ck, args.steps, args.warmup, True)
        if args.no_graph:
            ms_ck = ms_ck_e
        else:
            g_ck = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=True,
                                    form="checkpointed")
            ms_ck, _, _ = timed(g_ck.replay, args.steps, args.warmup, False)
        planes = (nsym + p.nx) * s * p.n_states
        checkpointed = {
            "value": T / (ms_ck * 1e-3), "unit": "time-steps/s", "ms_per_step": ms_ck,
            "eager_ms_per_step": round(ms_ck_e, 4),
            "outputs": "as the headline step: x*, P^s, log-likelihood, objective, adjoint",
            "kept_bytes": int(ck_out["ckpt"].numel()),
            "kept_bytes_saved_planes": int(planes),
            "kernels_ms": {k: round(v[1], 4) for k, v in kern_ck.items()},
            "kernels_note": "averages pool the forward call's and the adjoint's launches of "
                            "each kind (the adjoint's filter up-sweep skips the cross-block "
                            "step)"}

    res = {
        "metric": METRIC,
        "value": T / (ms_fa * 1e-3),
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_fa,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D constant-velocity SDE nx=4 ny=2, T=2^%d steps dt=1e-3, q=0.5, "
                               "r=0.05, one trajectory; filter + smoother (x*, P^s) + log-lik + "
                               "objective + adjoint d/d(gamma,q,r)" % args.log2T,
                   "T": T, "nx": 4, "ny": 2, "n_seg": 1, "storage": args.dtype,
                   "schedule": schedule_info(chunk, tuned)},
        "plain_scan": {"value": T / (ms_pl * 1e-3), "ms_per_step": ms_pl,
                       "kernels_ms": {k: round(v[1], 4) for k, v in kern_pl.items()}},
        "wall_ms_per_step": round(wall_fa, 4),
        "timing": "HIP-graph replay of the launch sequence" if not args.no_graph else "eager launches",
        "eager_ms_per_step": {"fwd_adjoint": round(ms_fa_e, 4), "plain": round(ms_pl_e, 4)},
        "roofline": roofline,
    }
    if two_filter is not None:
        res["two_filter"] = two_filter
    if fp32 is not None:
        res["fp32_storage"] = fp32
    if checkpointed is not None:
        res["checkpointed"] = checkpointed

    if args.copy_calibration:
        # plain device-to-device copy of a known size, read and written once,
        # and an FP64 multiply of a known number of elements (one flop each)
        nbytes = 256 << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        x = torch.full((1 << 24,), 1.5, dtype=torch.float64, device=dev)
        x.mul_(1.0000001)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = nbytes
        res["flop_calibration_fp64"] = 1 << 24
    ex_res = None
    if not args.no_exact:
        ex_res, wl_ex = measure_exact(args, ms, _lib, lib, timed, tdt, s, wl)
        res["exact_dynamics"] = ex_res
    ct_res = None
    if not args.no_ct:
        ct_res, wl_ct = measure_ct(args, ms, _lib, lib, timed, tdt, s)
        res["coordinated_turn"] = ct_res
    bt_res = None
    if not args.no_batched:
        bt_res, wl_bt = measure_batched(args, ms, _lib, lib, timed)
        res["batched"] = bt_res
    if not args.no_cpu_baseline:
        import tempfile

        from oracle import cref
        native = cref.native_lib(tempfile.mkdtemp(prefix="mapscan_oracle_"))
        res["cpu_baseline"] = cpu_baseline(wl, native, res["value"], res["plain_scan"]["value"],
                                           args.cpu_sample_steps, args.cpu_reps)
        if two_filter is not None:
            two_filter["cpu_baseline"] = cpu_baseline_two_filter(wl, args.cpu_sample_tf)
        if ct_res is not None:
            ct_res["cpu_baseline"] = cpu_baseline_ct(wl_ct, args.cpu_sample_ct, native)
        if ex_res is not None:
            ex_res["cpu_baseline"] = cpu_baseline_exact(wl_ex, args.cpu_sample_tf, native)
        if bt_res is not None:
            bt_res["cpu_baseline"] = cpu_baseline_batched(wl_bt, native, bt_res["value"],
                                                          args.cpu_batched_segs,
                                                          min(args.cpu_reps, 3))
    print(json.dumps(res))


def host_threads():
    """Threads for a CPU-baseline pool: the host CPUs this process may run on,
    capped at 16 (one GPU's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def timed_runs(fn, reps=5):
    """One untimed warm-up, then `reps` timed runs: (median, mean, all) seconds."""
    import statistics
    fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), sum(ts) / len(ts), ts


def cpu_baseline(wl, native, gpu_fa, gpu_plain, n_autograd, reps=5):
    """The sequential C oracle, compiled for this host (gcc -O3 -march=native),
    over the whole workload (all T steps): covariance-form Kalman filter + RTS
    smoother with covariances + log-likelihood + objective, FP64, one thread;
    median of 5 timed runs after one warm-up.  It computes no gradients, so the
    fwd+adjoint speedup compares more GPU work with less CPU work.  Beside it,
    the PyTorch oracle with its gradients by autograd on a prefix."""
    import torch

    from oracle import cref, ref

    T = int(wl.n_steps)
    med, mean, ts = timed_runs(lambda: cref.smooth(wl, lib=native), reps)
    value = T / med
    torch.set_num_threads(1)
    sub = workloads_prefix(wl, n_autograd)
    seg = ref.workload_segment(sub, 0)
    t0 = time.perf_counter()
    ref.gradients("cv", 4, seg, torch.zeros(n_autograd + 1, 4, dtype=torch.float64))
    t_ag = time.perf_counter() - t0
    return {"value": value, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": "all %d steps of the workload: sequential C Kalman filter + RTS smoother + "
                      "log-likelihood + objective (no gradients), FP64, gcc -O3 -march=native, "
                      "median of %d runs after a warm-up (%.2f s each)" % (T, reps, med),
            "median_s": round(med, 4), "mean_s": round(mean, 4),
            "runs_s": [round(t, 4) for t in ts],
            "speedup_fwd_adjoint": round(gpu_fa / value, 1),
            "speedup_plain_scan": round(gpu_plain / value, 1),
            "nproc": os.cpu_count(), "cpu": cpu_info(),
            "autograd_oracle": {"value": n_autograd / t_ag, "unit": "time-steps/s", "cores": 1,
                                "sample": "first %d steps: PyTorch per-step Kalman filter + RTS + "
                                          "log-likelihood + objective with gradients by autograd, "
                                          "%.1f s" % (n_autograd, t_ag)}}


def measure_ct(args, ms, _lib, lib, timed, tdt, s):
    """The paper's nonlinear experiment (Sec. 5.2): coordinated-turn tracks,
    5 Gauss--Newton iterations from m0, each a full RTS-form solve; the last
    one also gives P^s, the log-likelihood and the objective."""
    import torch

    import workloads

    wl = workloads.ct()
    p = ms.problem_from_workload(wl, dtype=tdt, device="cuda:0", chunk=args.ct_chunk)
    if not args.no_autotune and args.ct_chunk == 0:
        # the autotuner times one linear solve: linearise about the simulated path
        p.set_xbar(torch.as_tensor(wl.x_true))
        ms.autotune(p)
    f64 = torch.float64
    out = dict(xbar=p._tiled(p.nx), S=p._tiled(p.nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx),
               Ps=p._tiled(p.nsym), loglik=p._empty(p.n_seg, dtype=f64),
               obj=p._empty(p.n_seg, dtype=f64))

    def step():
        ms.iterated_nonlinear(p, wl.n_iter, covariances=True, loglik=True, objective=True,
                              out=out, natural=False)

    ms_e, _, kern = timed(step, args.steps, args.warmup, True)
    if args.no_graph:
        ms_g = ms_e
    else:
        g = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=False,
                             form="iterated", n_iter=wl.n_iter)
        ms_g, _, _ = timed(g.replay, args.steps, args.warmup, False)
    rec, fresh = counter_record(args.dtype, "ct5_64x2p14")
    # per-launch averages pool the 5 iterations (the last with covariances)
    roof = roofline_for(kern, rec, fresh, p.n_states, p.nx, p.ny, s, args.dtype, ms.schedule(p))
    res = {"value": wl.n_steps / (ms_g * 1e-3), "unit": "time-steps/s",
           "ms_per_step": ms_g, "eager_ms_per_step": round(ms_e, 4),
           "workload": "coordinated-turn SDE (Sec. 5.2) nx=5 ny=2 (range, bearing), 64 tracks x "
                       "2^14 steps dt=1e-3, 5 Gauss-Newton iterations from m0; x*, P^s, "
                       "log-likelihood, objective of the last",
           "n_iter": wl.n_iter, "n_steps": wl.n_steps,
           "schedule": schedule_info(ms.schedule(p),
                                     not args.no_autotune and args.ct_chunk == 0),
           "roofline": roof}
    return res, wl


def measure_batched(args, ms, _lib, lib, timed):
    """Batched segmented scan: 4096 independent constant-velocity tracks of
    ragged lengths floor(2^U(8, 14)) (about 1.6e7 steps) in one launch
    sequence, FP32 storage; per-segment log-likelihood, objective and their
    gradients in (gamma, q, r), smoothed x*, P^s."""
    import torch

    import workloads

    wl = workloads.config(4).rounded("f32")
    p = ms.problem_from_workload(wl, dtype=torch.float32, device="cuda:0")
    if not args.no_autotune:
        ms.autotune(p)
    f64 = torch.float64
    n = p.n_seg
    out = dict(S=p._tiled(p.nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx), Ps=p._tiled(p.nsym),
               loglik=p._empty(n, dtype=f64), obj=p._empty(n, dtype=f64),
               g_loglik=p._empty(n, 3, dtype=f64), g_obj=p._empty(n, 3, dtype=f64))

    def step():
        ms.smooth(p, covariances=True, loglik=True, objective=True, grad=True, out=out,
                  natural=False)

    ms_e, _, kern = timed(step, args.steps, args.warmup, True)
    if args.no_graph:
        ms_g = ms_e
    else:
        g = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=True)
        ms_g, _, _ = timed(g.replay, args.steps, args.warmup, False)
    rec, fresh = counter_record("f32", "cv4_batched4096")
    res = {"value": wl.n_steps / (ms_g * 1e-3), "unit": "time-steps/s", "ms_per_step": ms_g,
           "eager_ms_per_step": round(ms_e, 4),
           "workload": "4096 independent 2-D constant-velocity tracks, lengths "
                       "floor(2^U(8,14)) steps (%d steps in all), q ~ U[0.1,1], r ~ U[0.01,0.2], "
                       "dt=1e-3, FP32 storage; per-segment x*, P^s, log-likelihood, objective "
                       "and adjoint d/d(gamma,q,r)" % wl.n_steps,
           "n_seg": int(n), "n_steps": int(wl.n_steps), "storage": "f32",
           "schedule": schedule_info(ms.schedule(p), not args.no_autotune),
           "roofline": roofline_for(kern, rec, fresh, p.n_states, p.nx, p.ny, 4, "f32",
                                     ms.schedule(p))}
    return res, wl


def cpu_baseline_batched(wl, native, gpu_value, n_segs=1024, reps=3):
    """The sequential C oracle (gcc -O3 -march=native; covariance Kalman
    filter + RTS smoother + likelihood + objective, no gradients): one thread
    on the first n_segs segments, and a thread pool over contiguous groups of
    all segments on the host's threads (the C call releases the interpreter
    lock); median of `reps` runs after a warm-up each."""
    import concurrent.futures as cf

    from oracle import cref

    one = segment_range(wl, 0, n_segs) if 0 < n_segs < wl.n_seg else wl
    n1 = int(one.n_steps)
    med1, mean1, _ = timed_runs(lambda: cref.smooth(one, lib=native), reps)
    nt = host_threads()
    bounds = np.linspace(0, wl.n_seg, 4 * nt + 1).astype(int)
    parts = [segment_range(wl, a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    n = int(wl.n_steps)
    with cf.ThreadPoolExecutor(nt) as ex:
        medp, meanp, _ = timed_runs(lambda: list(ex.map(lambda w: cref.smooth(w, lib=native),
                                                        parts)), reps)
    return {"value": n1 / med1, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the %d segments (%d steps): sequential C Kalman filter + RTS "
                      "smoother + log-likelihood + objective (no gradients), FP64, gcc -O3 "
                      "-march=native, median of %d runs (%.2f s)"
                      % (one.n_seg, wl.n_seg, n1, reps, med1),
            "median_s": round(med1, 4), "mean_s": round(mean1, 4),
            "speedup": round(gpu_value / (n1 / med1), 1),
            "all_cores": {"value": n / medp, "unit": "time-steps/s", "cores": nt,
                          "median_s": round(medp, 4), "mean_s": round(meanp, 4),
                          "speedup": round(gpu_value / (n / medp), 1),
                          "sample": "all %d segments (%d steps) in %d groups over %d threads"
                                    % (wl.n_seg, n, len(parts), nt)},
            "nproc": os.cpu_count(), "cpu": cpu_info()}


def segment_range(wl, a, b):
    """Segments a..b-1 of a batched workload as a workload of their own."""
    import workloads

    k0, k1 = int(wl.seg_off[a]), int(wl.seg_off[b])
    sub = workloads.Workload(**{**wl.__dict__})
    sub.seg_off = wl.seg_off[a:b + 1] - k0
    sub.dt = wl.dt[k0:k1] if len(wl.dt) > 1 else wl.dt
    sub.y = wl.y[:, k0:k1]
    sub.theta, sub.m0, sub.P0 = wl.theta[a:b], wl.m0[a:b], wl.P0[a:b]
    sub.x_true = wl.x_true[:, k0 + a:k1 + b]
    return sub


def exact_terms_cv(q, gamma=0.0):
    import numpy as np
    F = np.zeros((4, 4)); F[:2, 2:] = np.eye(2); F[2:, 2:] = -gamma * np.eye(2)
    L = np.vstack([np.zeros((2, 2)), np.eye(2)])
    return F, np.zeros(4), L, q * np.eye(2)


def measure_exact(args, ms, _lib, lib, timed, tdt, s, wl):
    """The same 2^20-step track with exact (Van Loan) dynamics in the elements
    (map_lti_exact_terms), run through the general linear model: filter,
    smoother with covariances, log-likelihood and objective."""
    import numpy as np
    import torch

    import workloads

    q, r, dt = 0.5, 0.05, float(wl.dt[0])
    Ft, ct, Lt, Wt = ms.lti_exact_terms(*exact_terms_cv(q), dt)
    lin = dict(F=Ft, c=ct, L=Lt, W=Wt, H=np.hstack([np.eye(2), np.zeros((2, 2))]),
               r=np.zeros(2), R=r * np.eye(2))
    wx = workloads.Workload(name="cv_exact", model="linear", nx=4, ny=2, nw=4, seg_off=wl.seg_off,
                            dt=wl.dt, y=wl.y, theta=np.zeros((1, 0)), m0=wl.m0, P0=wl.P0,
                            x_true=wl.x_true, lin=lin)
    # one step length for all steps: every term of the general linear model is
    # shared, so the kernels build a step's terms once per block
    import dataclasses
    assert np.all(wx.dt == wx.dt[0])
    p = ms.problem_from_workload(dataclasses.replace(wx, dt=np.asarray(float(wx.dt[0]))),
                                 dtype=tdt, device="cuda:0")
    if not args.no_autotune:
        ms.autotune(p)
    f64 = torch.float64
    out = dict(S=p._tiled(p.nsym), v=p._tiled(p.nx), xs=p._tiled(p.nx), Ps=p._tiled(p.nsym),
               loglik=p._empty(1, dtype=f64), obj=p._empty(1, dtype=f64))

    def step():
        ms.smooth(p, covariances=True, loglik=True, objective=True, out=out, natural=False)

    ms_e, _, kern = timed(step, args.steps, args.warmup, True)
    if args.no_graph:
        ms_g = ms_e
    else:
        g = ms.GraphedSmooth(p, covariances=True, loglik=True, objective=True, grad=False)
        ms_g, _, _ = timed(g.replay, args.steps, args.warmup, False)
    rec, fresh = counter_record(args.dtype, "lin4exact_T2p20")
    res = {"value": wx.n_steps / (ms_g * 1e-3), "unit": "time-steps/s", "ms_per_step": ms_g,
           "eager_ms_per_step": round(ms_e, 4),
           "workload": "the same 2-D constant-velocity track (T=2^20, dt=1e-3) with exact "
                       "(matrix-exponential) dynamics in the elements, general linear model "
                       "nx=4 ny=2 nw=4; x*, P^s, log-likelihood, objective",
           "schedule": schedule_info(ms.schedule(p), not args.no_autotune),
           "roofline": roofline_for(kern, rec, fresh, p.n_states, p.nx, p.ny, s, args.dtype,
                                     ms.schedule(p))}
    return res, wx


def cpu_baseline_exact(wx, n, native):
    """The plain-C sequential oracle (covariance Kalman filter + RTS smoother +
    likelihood + objective) on the oracle's own exact terms, first n steps."""
    import numpy as np

    from oracle import cref, lti

    q, r, dt = 0.5, 0.05, float(wx.dt[0])
    Ft, ct, Lt, Wt = lti.implicit_equivalent(*exact_terms_cv(q), dt)
    sub = workloads_prefix(wx, n)
    per = lambda m: np.broadcast_to(m, (n,) + m.shape)
    sub.lin = dict(F=per(Ft), c=per(ct), L=Lt, W=Wt, H=per(wx.lin["H"]), r=per(wx.lin["r"]),
                   R=wx.lin["R"])
    dt_, _, _ = timed_runs(lambda: cref.smooth(sub, lib=native), reps=3)
    return {"value": n / dt_, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d steps of the same track: sequential C Kalman filter + RTS "
                      "smoother + log-likelihood + objective on exact terms, FP64, gcc -O3 "
                      "-march=native, median of 3 runs (%.2f s)" % (n, dt_), "cpu": cpu_info()}


def first_tracks(wl, n):
    """The first n segments of a workload of equal-length segments."""
    import workloads

    T = int(wl.seg_off[1] - wl.seg_off[0])
    sub = workloads.Workload(**{**wl.__dict__})
    sub.seg_off = wl.seg_off[:n + 1].copy()
    sub.dt, sub.y = wl.dt[:n * T], wl.y[:, :n * T]
    sub.theta, sub.m0, sub.P0 = wl.theta[:n], wl.m0[:n], wl.P0[:n]
    sub.x_true = wl.x_true[:, :n * (T + 1)]
    return sub


def cpu_baseline_ct(wl, n_tracks, native):
    """The plain-C sequential oracle (covariance Kalman filter + RTS per
    iteration) running the same 5 iterations on the first n_tracks tracks,
    one thread."""
    from oracle import cref

    sub = first_tracks(wl, n_tracks)
    t0 = time.perf_counter()
    cref.iterate(sub, lib=native)
    dt = time.perf_counter() - t0
    n = int(sub.n_steps)
    return {"value": n / dt, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the 64 tracks (%d steps), 5 iterations of the sequential C "
                      "Kalman filter + RTS smoother, FP64, gcc -O3 -march=native, %.1f s"
                      % (n_tracks, n, dt), "cpu": cpu_info()}


def cpu_baseline_two_filter(wl, n):
    """The plain-C sequential oracle of the two-filter smoother (covariance
    Kalman filter, then the later-step runs by the combination rule and one
    joint solve per state) on the first n steps of the same trajectory, one
    thread."""
    from oracle import cref

    sub = workloads_prefix(wl, n)
    t0 = time.perf_counter()
    cref.two_filter(sub)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d steps of the same trajectory: sequential C two-filter smoother "
                      "(filter, later-step runs, per-state joint solve), FP64, %.1f s" % (n, dt),
            "cpu": cpu_info()}


def workloads_prefix(wl, n):
    import workloads

    sub = workloads.Workload(**{**wl.__dict__})
    sub.seg_off = wl.seg_off.copy()
    sub.seg_off[-1] = n
    sub.dt = wl.dt[:n]
    sub.y = wl.y[:, :n]
    sub.x_true = wl.x_true[:, :n + 1]
    return sub


if __name__ == "__main__":
    main()
